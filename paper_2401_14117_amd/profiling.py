"""Summaries of rocprofv3 output (a reporting utility): the Rgemm kernel's
time and HBM traffic, and per-kernel time tables of other traced commands.

rocprofv3 is run on the MI355X machine by the commands recorded in each summary;
this module only reads the CSV files it writes:

* ``<dir>/*_kernel_trace.csv`` (``--kernel-trace --output-format csv``):
  per-dispatch start/end timestamps, from which per-kernel call counts and
  average durations are taken;
* ``<dir>/*_counter_collection.csv`` (``--pmc ...``): per-dispatch counter
  values.  FETCH_SIZE and WRITE_SIZE are in KiB per dispatch.

HBM traffic of a kernel is FETCH_SIZE + WRITE_SIZE, each scaled by the ratio
between the known size of a plain device copy and what the same counter reads
for that copy (run under the same profiler in the same job).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os


WHERE = ("run on the MI355X box from /tmp, REPO = the repository root, "
         "OUT = the directory the profiler writes to")


def _one(d: str, suffix: str) -> str:
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return sorted(files)[0]


def kernel_stats(trace_dir: str) -> dict:
    """name -> (calls, average duration in ns) from a kernel trace."""
    acc = collections.defaultdict(list)
    with open(_one(trace_dir, "_kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            acc[r["Kernel_Name"]].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def counter_per_dispatch(pmc_dir: str, counter: str, match: str) -> float:
    """Average per-dispatch value of a counter over dispatches of kernels
    whose name contains `match`."""
    per = collections.defaultdict(float)
    with open(_one(pmc_dir, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter and match in r["Kernel_Name"]:
                per[r["Dispatch_Id"]] += float(r["Counter_Value"])
    if not per:
        raise ValueError(f"no {counter} samples for kernels matching {match!r}")
    return sum(per.values()) / len(per)


def summarize(args) -> None:
    stats = kernel_stats(args.trace)
    copy_bytes = args.copy_bytes
    fetch_f = copy_bytes / (1024.0 * counter_per_dispatch(args.copy_fetch, "FETCH_SIZE", args.copy_kernel))
    write_f = copy_bytes / (1024.0 * counter_per_dispatch(args.copy_write, "WRITE_SIZE", args.copy_kernel))
    fetch_kib = counter_per_dispatch(args.fetch, "FETCH_SIZE", args.kernel)
    write_kib = counter_per_dispatch(args.write, "WRITE_SIZE", args.kernel)
    hbm = fetch_kib * 1024 * fetch_f + write_kib * 1024 * write_f
    name = next(k for k in stats if args.kernel in k)
    calls, avg_ns = stats[name]
    m, n, k = args.mnk
    algo = 4 * (m * k + k * n + 2 * m * n)
    lines = [
        f"# rocprofv3: Posit(32,2) Rgemm kernel, {args.workload}",
        "",
        f"Kernel: `{name}`",
        f"Workload: {args.workload} (m = {m}, n = {n}, k = {k}).",
        f"Kernel source hash: {args.kernel_hash}.",
        "",
        "Commands (" + WHERE + "):",
        "",
        "```",
        f"rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/trace -o trace -- "
        f"python3 $REPO/bench.py --workload {args.workload} --steps 2 --warmup 1 --cpu-budget 0 --extras 0",
        f"rocprofv3 --pmc FETCH_SIZE --kernel-trace --output-format csv -d $OUT/fetch -o fetch -- "
        f"python3 $REPO/bench.py --workload {args.workload} --steps 1 --warmup 0 --cpu-budget 0 --extras 0",
        f"rocprofv3 --pmc WRITE_SIZE --kernel-trace --output-format csv -d $OUT/write -o write -- "
        f"python3 $REPO/bench.py --workload {args.workload} --steps 1 --warmup 0 --cpu-budget 0 --extras 0",
        "rocprofv3 --pmc FETCH_SIZE --kernel-trace --output-format csv -d $OUT/copyf -o copyf -- "
        "python3 $REPO/bench.py --copy-calibration",
        "rocprofv3 --pmc WRITE_SIZE --kernel-trace --output-format csv -d $OUT/copyw -o copyw -- "
        "python3 $REPO/bench.py --copy-calibration",
        "```",
        "",
        "| quantity | value |",
        "|---|---|",
        f"| kernel calls (trace run) | {calls} |",
        f"| average kernel duration | {avg_ns / 1e6:.3f} ms |",
        f"| Gpops/s from the trace (2mnk / duration) | {2.0 * m * n * k / avg_ns:.1f} |",
        f"| FETCH_SIZE per dispatch | {fetch_kib:.0f} KiB |",
        f"| WRITE_SIZE per dispatch | {write_kib:.0f} KiB |",
        f"| copy calibration ({copy_bytes >> 20} MiB copy): fetch factor | {fetch_f:.3f} |",
        f"| copy calibration: write factor | {write_f:.3f} |",
        f"| HBM traffic per dispatch (scaled) | {hbm / 1e9:.3f} GB |",
        f"| algorithmic bytes 4(mk + kn + 2mn) | {algo / 1e9:.3f} GB |",
        f"| HBM bandwidth used | {hbm / (avg_ns * 1e-9) / 1e9:.1f} GB/s (of 8000) |",
    ]
    others = sorted(((v[1] * v[0], k, v) for k, v in stats.items() if k != name), reverse=True)[:4]
    if others:
        lines += ["", "Other kernels in the traced run (setup: conversions, masks, copies):", ""]
        for _, kname, (c, a) in others:
            short = kname if len(kname) < 80 else kname[:77] + "..."
            lines.append(f"- `{short}`: {c} calls, {a / 1e3:.1f} us average")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    if args.traffic_json:
        data = {}
        if os.path.exists(args.traffic_json):
            with open(args.traffic_json) as f:
                data = json.load(f)
        data[args.workload] = {"kernel_hash": args.kernel_hash, "hbm_bytes_per_launch": round(hbm),
                               "fetch_kib": fetch_kib, "write_kib": write_kib,
                               "fetch_factor": fetch_f, "write_factor": write_f,
                               "avg_kernel_ms": avg_ns / 1e6}
        with open(args.traffic_json, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


def kernel_table(args) -> None:
    """Per-kernel calls, total and average time of one traced command."""
    stats = kernel_stats(args.trace)
    rows = sorted(((c * a, k, c, a) for k, (c, a) in stats.items()), reverse=True)
    total = sum(r[0] for r in rows)
    lines = [f"# rocprofv3: {args.title}", "", "Command (" + WHERE + "):", "", "```", args.command, "```", "",
             f"Kernel time in the traced run: {total / 1e6:.2f} ms.", "",
             "| kernel | calls | total ms | average us | share |", "|---|---|---|---|---|"]
    for tot, k, c, a in rows[:args.top]:
        short = k if len(k) < 90 else k[:87] + "..."
        lines.append(f"| `{short}` | {c} | {tot / 1e6:.2f} | {a / 1e3:.1f} | {tot / total:.1%} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def valu_table(args) -> None:
    """VALU utilisation of the Rgemm kernel from one SQ counter pass: VALU
    instructions per multiply-add and the issue rate against the chip's
    integer-VALU peaks (256 CUs x 2.4 GHz x 128 or 64 lanes per clock)."""
    stats = kernel_stats(args.trace)
    name = next(k for k in stats if args.kernel in k)
    avg_ns = stats[name][1]
    m, n, k = args.mnk
    madds = float(args.madds) if args.madds else float(m) * n * k
    ctr = {c: counter_per_dispatch(args.pmc, c, args.kernel) for c in args.counters}
    cycles = avg_ns * 1e-9 * args.clock_ghz * 1e9
    bench_args = args.bench_args or f"--workload {args.workload} --steps 1 --warmup 0 --cpu-budget 0 --extras 0"
    lines = [f"# rocprofv3: VALU utilisation of the {args.what}, {args.workload}", "",
             f"Kernel: `{name}`", f"Kernel source hash: {args.kernel_hash}.", "",
             "Commands (" + WHERE + "):", "", "```",
             f"rocprofv3 --pmc {' '.join(args.counters)} --kernel-trace --output-format csv "
             f"-d $OUT/valu -o valu -- python3 $REPO/bench.py {bench_args}",
             f"(kernel duration from the --kernel-trace --stats run: {args.trace_note})", "```", "",
             f"Multiply-adds per dispatch: {madds:.4g}" + (f" ({args.madds_note})" if args.madds_note else "") + ".",
             "",
             "| counter (per dispatch, summed over the chip) | value |", "|---|---|"]
    for c in args.counters:
        lines.append(f"| {c} | {ctr[c]:.4g} |")
    lines += ["", "| derived | value |", "|---|---|",
              f"| average kernel duration (trace) | {avg_ns / 1e6:.3f} ms |"]
    if "SQ_INSTS_VALU" in ctr:
        lane = ctr["SQ_INSTS_VALU"] * 64.0
        rate = lane / (avg_ns * 1e-9)
        per_cu = ctr["SQ_INSTS_VALU"] / args.cus / cycles
        lines += [f"| VALU lane-instructions per multiply-add (whole kernel) | {lane / madds:.2f} |",
                  f"| VALU issue rate | {rate / 1e12:.2f} T lane-instr/s |",
                  f"| of the 128-lane/clk/CU peak ({args.cus * 128 * args.clock_ghz / 1e3:.1f} T) | "
                  f"{rate / (args.cus * 128 * args.clock_ghz * 1e9):.1%} |",
                  f"| of the 64-lane/clk/CU rate ({args.cus * 64 * args.clock_ghz / 1e3:.1f} T) | "
                  f"{rate / (args.cus * 64 * args.clock_ghz * 1e9):.1%} |",
                  f"| wave-instructions per CU per clock | {per_cu:.3f} |"]
    if "SQ_INSTS_LDS" in ctr:
        lines.append(f"| LDS instructions per multiply-add (per 64 lanes) | {ctr['SQ_INSTS_LDS'] * 64 / madds:.3f} |")
    if "SQ_INSTS_SALU" in ctr:
        lines.append(f"| SALU instructions per multiply-add (per 64 lanes) | {ctr['SQ_INSTS_SALU'] * 64 / madds:.3f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main() -> None:
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "valu":
        ap = argparse.ArgumentParser(description=valu_table.__doc__)
        ap.add_argument("mode")
        ap.add_argument("--trace", required=True)
        ap.add_argument("--pmc", required=True)
        ap.add_argument("--counters", nargs="+", required=True)
        ap.add_argument("--kernel", default="gemm_kernel<false, false, false, false>")
        ap.add_argument("--workload", default="square_n8192")
        ap.add_argument("--mnk", type=int, nargs=3, default=[8192, 8192, 8192])
        ap.add_argument("--cus", type=int, default=256)
        ap.add_argument("--clock-ghz", type=float, default=2.4)
        ap.add_argument("--kernel-hash", required=True)
        ap.add_argument("--out", required=True)
        ap.add_argument("--what", default="Posit(32,2) Rgemm kernel")
        ap.add_argument("--madds", type=float, default=0.0, help="multiply-adds per dispatch (default m n k)")
        ap.add_argument("--madds-note", default="")
        ap.add_argument("--bench-args", default="")
        ap.add_argument("--trace-note", default="the Rgemm summary")
        valu_table(ap.parse_args())
        return
    if len(sys.argv) > 1 and sys.argv[1] == "kernels":
        ap = argparse.ArgumentParser(description=kernel_table.__doc__)
        ap.add_argument("mode")
        ap.add_argument("--trace", required=True)
        ap.add_argument("--title", required=True)
        ap.add_argument("--command", required=True)
        ap.add_argument("--top", type=int, default=12)
        ap.add_argument("--out", required=True)
        kernel_table(ap.parse_args())
        return
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--copy-kernel", default="copyBuffer")
    ap.add_argument("--kernel", default="gemm_kernel<false, false, false, false>")
    ap.add_argument("--workload", default="square_n8192")
    ap.add_argument("--mnk", type=int, nargs=3, default=[8192, 8192, 8192])
    ap.add_argument("--kernel-hash", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic-json")
    summarize(ap.parse_args())


if __name__ == "__main__":
    main()
