#!/usr/bin/env python3
"""Benchmark of the Posit(32,2) Rgemm hot path on one MI355X.

One step = one C = alpha*A*B + beta*C call of the HIP library (posit32_gemm)
over the whole synthetic workload, inputs already resident in HBM.  The
default workload is the square n = 8192 case of the Rgemm sweep (magnitudes
uniform[-1,1] * 2^s, s in [-12,12], NaR/zero sprinkle 1e-6, alpha = beta = 1).

Prints ONE JSON line with the metric, the roofline of the Rgemm kernel
(integer-VALU bound) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Integer VALU ceiling: 256 CUs x 128 lane-ops per clock x 2.4 GHz = 78.6 T
# lane-ops/s.  128 lanes/clk/CU is the rate at which gfx950 retires the simple
# 32-bit integer ops (add, sub, and, or, xor, shifts right, mov) when two can
# issue together, the same lane rate as the chip's FP32 vector peak
# (157.3 TFLOP/s = 78.6 T FMA/s); other VALU ops retire at 64 lanes/clk/CU.
PEAK_INT_TOPS = 256 * 128 * 2.4e9 / 1e12
PKG = os.path.join(ROOT, "paper_2401_14117_amd")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("p32_device.hpp", "p32_gemm_tile.hpp", "p32_gemm.hip"):
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_valu_per_madd() -> float | None:
    """Fast-path VALU instructions per multiply-add of the built kernel, counted
    from its ISA when the library was built."""
    path = os.path.join(PKG, "libposit32.isa.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        info = json.load(f)
    if info.get("kernel_hash") != kernel_source_hash():
        return None
    return float(info["valu_per_madd"])


def load_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "gemm_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        info = json.load(f)
    rec = info.get(workload)
    if not rec or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def make_case(name: str):
    from paper_2401_14117_amd import workloads as W
    if name.startswith("square_n"):
        return W.gemm_square(int(name[len("square_n"):]))
    if name.startswith("trailing_j"):
        return W.gemm_trailing(int(name[len("trailing_j"):]))
    if name.startswith("uniform_n"):
        n = int(name[len("uniform_n"):])
        return W.gemm_uniform(n, n, n, seed=1)
    if name.startswith("normal_sigma"):           # normal_sigma<S>_n<N>
        sig, n = name[len("normal_sigma"):].split("_n")
        return W.gemm_normal(int(n), float(sig))
    raise SystemExit(f"unknown workload {name}")


STREAM_PROCESSORS = 256 * 64      # MI355X: 256 CUs x 64 lanes
EW_OPS = {"add": 0, "mul": 2, "div": 3, "sqrt": 4}


def run_elementwise_bench(name: str, args, dev) -> dict:
    """ew_<op>_<range>: the paper's elementwise kernel study (Section 4.2,
    Table 2) -- n operations on arrays p, q drawn from one magnitude range.
    One step = one posit32_elementwise launch over the whole arrays."""
    import torch
    from paper_2401_14117_amd import posit32
    from paper_2401_14117_amd import workloads as W
    _, op_name, rng_name = name.split("_")
    op = EW_OPS[op_name]
    n = args.ew_n
    p, q = W.elementwise_range(n, rng_name)
    P = posit32.from_f64(torch.from_numpy(p).to(dev))
    Q = posit32.from_f64(torch.from_numpy(q).to(dev))
    out = torch.empty_like(P)
    stream = torch.cuda.current_stream()

    def step(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        posit32.elementwise(op, P, None if op == 4 else Q, out=out)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        step(e0, e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    nbytes = n * (8 if op == 4 else 12)
    return {
        "metric": f"Posit32 elementwise {op_name} Gop/s ({rng_name})",
        "value": round(n / (kms * 1e-3) / 1e9, 2),
        "unit": "Gop/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "posit32 (int32 VALU)",
        "data": "synthetic",
        "config": {"workload": name, "n": n, "range": list(W.RANGES[rng_name]),
                   "kernel_ms": round(kms, 4),
                   "ns_per_op_per_stream_processor": round(kms * 1e6 * STREAM_PROCESSORS / n, 2)},
        "roofline": {"bound": "hbm", "achieved": round(nbytes / (kms * 1e-3) / 1e9, 1),
                     "peak": 8000.0, "unit": "GB/s",
                     "frac": round(nbytes / (kms * 1e-3) / 1e9 / 8000.0, 4), "traffic": None},
        "cpu_baseline": None,
    }


def _socket_power_w() -> float | None:
    """GPU package power in watts as amd-smi reports it (None when unavailable)."""
    try:
        out = subprocess.run(["amd-smi", "metric", "-p"], capture_output=True, text=True,
                             timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    m = re.search(r"SOCKET_POWER:\s*([0-9.]+)\s*W", out)
    return float(m.group(1)) if m else None


def _power_while(step, seconds: float) -> dict | None:
    """Mean GPU package power while `step` runs back to back for `seconds`
    (amd-smi sampled from a second thread), with the idle reading before."""
    import torch
    idle = _socket_power_w()
    if idle is None or seconds <= 0:
        return None
    samples, stop = [], threading.Event()

    def sampler():
        while not stop.is_set():
            w = _socket_power_w()
            if w is not None:
                samples.append(w)
            stop.wait(0.2)

    th = threading.Thread(target=sampler, daemon=True)
    th.start()
    t_end, runs = time.perf_counter() + seconds, 0
    while time.perf_counter() < t_end:
        step()
        torch.cuda.synchronize()
        runs += 1
    stop.set()
    th.join()
    # the first sample may predate the load
    busy = samples[1:] if len(samples) > 2 else samples
    if not busy:
        return None
    return {"socket_w_idle": idle, "socket_w_mean": round(float(np.mean(busy)), 1),
            "samples": len(busy), "runs": runs, "seconds": seconds}


def run_solve_bench(name: str, args, dev) -> dict:
    """Factor + solve workloads (getrf_nN / potrf_nN): one step = copy the
    matrix into the work buffer, factor it, solve A x = b (nrhs = 1)."""
    import torch
    from paper_2401_14117_amd import posit32
    from paper_2401_14117_amd import workloads as W
    kind, n = name.split("_n")
    n = int(n)
    case = W.lu_case(n) if kind == "getrf" else W.chol_case(n)
    A0 = posit32.from_f64(torch.from_numpy(case.A).to(dev))
    b0 = posit32.from_f64(torch.from_numpy(np.ascontiguousarray(case.b)).to(dev))
    A = torch.empty_like(A0)
    b = torch.empty_like(b0)
    stream = torch.cuda.current_stream()

    def step(ev0=None, ev1=None):
        A.copy_(A0)
        b.copy_(b0)
        if ev0 is not None:
            ev0.record(stream)
        if kind == "getrf":
            _, ipiv, info = posit32.getrf(A, args.nb)
            posit32.getrs(A, ipiv, b)
        else:
            _, info = posit32.potrf(A, args.nb)
            posit32.potrs(A, b)
        if ev1 is not None:
            ev1.record(stream)
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        info = step(e0, e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    pops = (2.0 if kind == "getrf" else 1.0) * n ** 3 / 3.0
    ms_per_step = wall * 1e3 / args.steps
    # accuracy of the solve (outside the timed region): forward error against
    # an FP64 solve, beside LAPACK binary32 (sgetrs/spotrs) on the same data
    import scipy.linalg as sl
    x = posit32.to_f64(b).cpu().numpy()[:, 0]
    x64 = np.linalg.solve(case.A, case.b[:, 0])
    if kind == "getrf":
        x32 = sl.lu_solve(sl.lu_factor(case.A.astype(np.float32)), case.b[:, 0].astype(np.float32))
    else:
        x32 = sl.cho_solve(sl.cho_factor(case.A.astype(np.float32), lower=True),
                           case.b[:, 0].astype(np.float32))
    err = float(np.linalg.norm(x - x64) / np.linalg.norm(x64))
    err32 = float(np.linalg.norm(x32.astype(np.float64) - x64) / np.linalg.norm(x64))
    # where the time goes (outside the timed region): the factorisation's
    # phases timed by HIP events between its launches (LU), then the solve
    A.copy_(A0)
    b.copy_(b0)
    torch.cuda.synchronize()
    phases = None
    if kind == "getrf":
        _, ipiv, _, phases = posit32.getrf_phases(A, args.nb)
    else:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        posit32.potrf(A, args.nb)
        e1.record(stream)
        torch.cuda.synchronize()
        phases = {"factor": round(e0.elapsed_time(e1), 3)}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    if kind == "getrf":
        posit32.getrs(A, ipiv, b)
    else:
        posit32.potrs(A, b)
    e1.record(stream)
    torch.cuda.synchronize()
    phases["solve"] = round(e0.elapsed_time(e1), 3)
    value = pops / (ms_per_step * 1e-3) / 1e9
    # GPU package power over repeated factor + solve runs (after the timed
    # region); the paper's LU figure is whole-system AC power, so it is context
    power = _power_while(step, args.power_seconds)
    if power is not None:
        power["source"] = "amd-smi metric -p, SOCKET_POWER (GPU package only)"
        power["gpops_per_w"] = round(value / power["socket_w_mean"], 3)
        if kind == "getrf":
            power["paper_lu_gflops_per_w"] = ("0.043-0.076: whole-system AC power, LU at N = 8000 on "
                                              "an FPGA and three GPUs (Sec. 5.3, Table 6)")
    return {
        "metric": f"Posit32 R{kind} + R{kind[:3]}rs Gpops/s (factor {'2' if kind == 'getrf' else '1'}n^3/3 pops)",
        "value": round(value, 3),
        "unit": "Gpops/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "posit32 (int32 VALU)", "data": "synthetic",
        "config": {"workload": case.name, "n": n, "nb": args.nb, "nrhs": 1,
                   "factor_solve_ms_events": round(kms, 3), "info": int(info.cpu().item()),
                   "forward_error_posit32": err, "forward_error_binary32": err32,
                   "digits_gained_vs_binary32": round(float(np.log10(err32 / err)), 3),
                   "phases_ms": phases, "power": power},
        "roofline": None, "cpu_baseline": None,
    }


def run_batch_bench(name: str, args, dev) -> dict:
    """batch_lu / batch_chol: the variable-size batched workload -- count
    systems (n log-uniform in [16, 512], nrhs in [1, 16]) factored and solved
    by one launch of one workgroup per system (posit32_gesv_vbatched /
    posit32_posv_vbatched).  One step = the whole batch, inputs resident in
    HBM (restored between steps outside the timed region).  Beside it: the
    same library's single-matrix calls, one system at a time, on a random
    sample of the batch (their results are also compared with the batched
    ones bit for bit)."""
    import torch
    from paper_2401_14117_amd import posit32
    from paper_2401_14117_amd import workloads as W
    kind = "lu" if name == "batch_lu" else "chol"
    n, nrhs = W.batch_sizes(args.batch_count)
    count = len(n)
    t0 = time.perf_counter()
    offA = np.concatenate([[0], np.cumsum(n * n)])
    offB = np.concatenate([[0], np.cumsum(n * nrhs)])
    A0 = torch.empty(int(offA[-1]), dtype=torch.int32, device=dev)
    B0 = torch.empty(int(offB[-1]), dtype=torch.int32, device=dev)
    pend_a, pend_b, first = [], [], 0
    flushed = 0

    def flush(upto):
        nonlocal pend_a, pend_b, first
        if not pend_a:
            return
        a = torch.from_numpy(np.concatenate(pend_a)).to(dev)
        b = torch.from_numpy(np.concatenate(pend_b)).to(dev)
        posit32.from_f64(a, out=A0[int(offA[first]):int(offA[upto])])
        posit32.from_f64(b, out=B0[int(offB[first]):int(offB[upto])])
        pend_a, pend_b, first = [], [], upto

    for i, A, B in W.batch_matrices(kind, n, nrhs):
        pend_a.append(A.ravel())
        pend_b.append(B.ravel())
        flushed += A.size
        if flushed >= (32 << 20):
            flush(i + 1)
            flushed = 0
    flush(count)
    A = A0.clone()
    B = B0.clone()
    order = np.argsort(-n, kind="stable")          # decreasing n balances the workgroups
    As = [A[int(offA[i]):int(offA[i + 1])].view(int(n[i]), int(n[i])) for i in order]
    Bs = [B[int(offB[i]):int(offB[i + 1])].view(int(n[i]), int(nrhs[i])) for i in order]
    vb = posit32.VBatch(As, Bs, lu=(kind == "lu"))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()

    def launch():
        if kind == "lu":
            vb.gesv(args.nb)
        else:
            vb.posv(args.nb)

    # the eager launch once (the reference for the graph's results), then the
    # launch captured in a hipGraph; each timed step replays the graph
    A.copy_(A0)
    B.copy_(B0)
    launch()
    torch.cuda.synchronize()
    eager_B, eager_info = B.clone(), vb.info.clone()
    A.copy_(A0)
    B.copy_(B0)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        launch()
    torch.cuda.synchronize()

    def step(ev0=None, ev1=None):
        A.copy_(A0)
        B.copy_(B0)
        if ev0 is not None:
            ev0.record(stream)
        graph.replay()
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for e0, e1 in evs:
        step(e0, e1)
    torch.cuda.synchronize()
    kms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    info = vb.info.cpu().numpy()
    graph_same = bool(torch.equal(B, eager_B) and torch.equal(vb.info, eager_info))
    fac = (2.0 if kind == "lu" else 1.0) / 3.0
    pops = float(np.sum(fac * n.astype(np.float64) ** 3))

    # one system at a time through the single-matrix entry points, on a sample
    if args.single_count <= 0:
        return _batch_result(name, kind, count, kms, pops, info, setup_s, None, None, args, graph_same)
    rs = np.random.default_rng(6001)
    sample = np.sort(rs.choice(count, size=min(args.single_count, count), replace=False))
    A.copy_(A0)
    B.copy_(B0)
    torch.cuda.synchronize()
    views = [(A[int(offA[i]):int(offA[i + 1])].view(int(n[i]), int(n[i])),
              B[int(offB[i]):int(offB[i + 1])].view(int(n[i]), int(nrhs[i]))) for i in sample]
    t1 = time.perf_counter()
    for Ai, Bi in views:
        if kind == "lu":
            _, ipiv, _ = posit32.getrf(Ai, args.nb)
            posit32.getrs(Ai, ipiv, Bi)
        else:
            posit32.potrf(Ai, args.nb)
            posit32.potrs(Ai, Bi)
    torch.cuda.synchronize()
    single_s = time.perf_counter() - t1
    single = {"sample": len(sample), "seconds": round(single_s, 3),
              "solves_per_s": round(len(sample) / single_s, 1),
              "sample_pops_share": round(float(np.sum(fac * n[sample].astype(np.float64) ** 3)) / pops, 5)}
    # bit-compare the sampled single-matrix results with the batched ones
    A_single = torch.cat([A[int(offA[i]):int(offA[i + 1])] for i in sample])
    B_single = torch.cat([B[int(offB[i]):int(offB[i + 1])] for i in sample])
    A.copy_(A0)
    B.copy_(B0)
    vb.gesv(args.nb) if kind == "lu" else vb.posv(args.nb)
    torch.cuda.synchronize()
    A_b = torch.cat([A[int(offA[i]):int(offA[i + 1])] for i in sample])
    B_b = torch.cat([B[int(offB[i]):int(offB[i + 1])] for i in sample])
    single["bit_identical_to_batched"] = bool(torch.equal(A_single, A_b) and torch.equal(B_single, B_b))
    # expected ratio if the single calls ran the whole batch: scale by work share
    single["whole_batch_s_est"] = round(single_s / max(single["sample_pops_share"], 1e-12), 2)

    cpu = None
    if args.cpu_budget > 0:
        import oracle as O
        done, tcpu = 0, time.perf_counter()
        for i, Af, Bf in W.batch_matrices(kind, n, nrhs, start=0, stop=count):
            Ap = O.vec_from_double(Af)
            Bp = O.vec_from_double(Bf)
            if kind == "lu":
                LU, ipiv, _ = O.getrf(Ap, args.nb)
                O.getrs(LU, ipiv, Bp)
            else:
                L, _ = O.potrf(Ap, args.nb)
                O.potrs(L, Bp)
            done += 1
            if time.perf_counter() - tcpu > args.cpu_budget:
                break
        el = time.perf_counter() - tcpu
        cpu = {"value": round(done / el, 3), "unit": "solves/s", "cores": O.num_threads(),
               "kind": "oracle", "sample": f"first {done} systems of the batch (in generation order)"}

    return _batch_result(name, kind, count, kms, pops, info, setup_s, single, cpu, args, graph_same)


def _tuning_info(kind: str) -> dict:
    """The sub-panel table the batched kernels ran with, and where it came from."""
    from paper_2401_14117_amd import posit32
    t = posit32.active_tuning(kind)
    src = posit32.tuning_file() if t is not None else "built-in"
    t = t if t is not None else posit32.default_tuning(kind)
    return {"source": os.path.relpath(src, ROOT) if src != "built-in" else src, **t.to_dict()}


def _batch_roofline(kind: str, kms: float, pops: float) -> dict | None:
    """Integer-VALU roofline of the batched kernel: the VALU lane-instructions
    per multiply-add measured by the committed SQ-counter summary of the
    same workload, times this run's multiply-adds (factor pops / 2) over this
    run's kernel time, against the 78.6 T lane-op/s peak."""
    path = os.path.join(ROOT, "profiles", f"batch_{kind}_valu_rocprof.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"VALU lane-instructions per multiply-add \(whole kernel\) \| ([0-9.]+) \|", open(path).read())
    if not m:
        return None
    per = float(m.group(1))
    achieved = per * (pops / 2.0) / (kms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_INT_TOPS, 2),
            "unit": "Tlane-op/s", "frac": round(achieved / PEAK_INT_TOPS, 4), "traffic": None,
            "valu_per_madd": per, "valu_per_madd_source": os.path.relpath(path, ROOT)}


def _batch_result(name, kind, count, kms, pops, info, setup_s, single, cpu, args, graph_same) -> dict:
    return {
        "metric": f"Posit32 batched {'LU' if kind == 'lu' else 'Cholesky'} factor+solve solves/s",
        "value": round(count / (kms * 1e-3), 1),
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(kms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "posit32 (int32 VALU)", "data": "synthetic",
        "config": {"workload": name, "count": count, "n": "round(exp(U(ln 16, ln 512)))",
                   "nrhs": "1..16", "nb": args.nb, "factor_gpops": round(pops / (kms * 1e-3) / 1e9, 1),
                   "info_nonzero": int(np.count_nonzero(info)), "setup_s": round(setup_s, 1),
                   "sub_panel_tuning": _tuning_info(kind),
                   "launch": "one kernel (a workgroup per system) captured in a hipGraph; each step is a replay",
                   "graph_bit_identical_to_eager": graph_same, "one_at_a_time": single},
        "roofline": _batch_roofline(kind, kms, pops),
        "cpu_baseline": cpu,
    }


def run_serve_bench(args, dev, kind: str = "lu") -> list[dict]:
    """serve_lu / serve_chol: the request queue under Poisson arrivals, one
    JSON line per arrival rate.  Each request is a new LU (or Cholesky) system
    (n log-uniform in [32, 2048], nrhs in [1, 32]); its latency is completion
    minus submission on the queue's own clock.  Payloads are converted to
    posit patterns before the clock starts; requests of the same n share one
    system (B's first nrhs columns)."""
    import threading
    import torch
    from paper_2401_14117_amd import posit32
    from paper_2401_14117_amd import workloads as W
    lines = []
    payload = {}                                   # n -> (A, B with 32 columns)
    req = posit32.REQ_LU if kind == "lu" else posit32.REQ_CHOL
    for qps in args.qps:
        t_arr, n, nrhs = W.serve_stream(qps, args.serve_seconds)
        for k in n.tolist():
            if k not in payload:
                A, B = W.serve_system(k, 32, 7000, kind)
                Ap = posit32.from_f64(torch.from_numpy(A).to(dev)).cpu().numpy().view(np.uint32)
                Bp = posit32.from_f64(torch.from_numpy(B).to(dev)).cpu().numpy().view(np.uint32)
                payload[k] = (Ap, Bp)
        q = posit32.Queue(device_bytes=8 << 30, max_batch=1024, nb=args.nb, batch_max_n=args.batch_max_n)
        # warm-up: one small and one large system
        for k in (64, 1024):
            A, B = W.serve_system(k, 2, 7001, kind)
            Ap = posit32.from_f64(torch.from_numpy(A).to(dev)).cpu().numpy().view(np.uint32)
            Bp = posit32.from_f64(torch.from_numpy(B).to(dev)).cpu().numpy().view(np.uint32)
            q.wait(q.submit(req, Bp, Ap), 120.0)
        tickets = [None] * len(n)
        t0 = time.perf_counter()

        def submitter():
            for i in range(len(n)):
                delay = t_arr[i] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                Ap, Bp = payload[int(n[i])]
                tickets[i] = q.submit(req, Bp[:, :int(nrhs[i])], Ap)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        outs = [q.wait(t, 600.0) for t in tickets]
        st = q.stats()
        q.close()
        single = _serve_burst_vs_one_at_a_time(payload, n, nrhs, outs, args, dev, kind) \
            if qps == args.qps[-1] else None
        lat = np.array([o["done_s"] - o["submit_s"] for o in outs]) * 1e3
        span = max(o["done_s"] for o in outs) - min(o["submit_s"] for o in outs)
        bad = sum(1 for o in outs if o["status"] != 0 or o["info"] != 0)
        small = n <= 512
        lines.append({
            "metric": f"Posit32 served {'LU' if kind == 'lu' else 'Cholesky'} factor+solve solves/s "
                      "(Poisson arrivals, p50/p99 latency)",
            "value": round(len(n) / span, 1), "unit": "solves/s", "n_gpus": 1,
            "steps": 1, "warmup": 2, "ms_per_step": round(span * 1e3, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "posit32 (int32 VALU)",
            "data": "synthetic",
            "config": {"workload": f"serve_{kind}", "qps": qps, "requests": int(len(n)),
                       "seconds": args.serve_seconds, "n": "round(exp(U(ln 32, ln 2048)))",
                       "nrhs": "1..32", "batch_max_n": args.batch_max_n,
                       "p50_ms": round(float(np.percentile(lat, 50)), 2),
                       "p99_ms": round(float(np.percentile(lat, 99)), 2),
                       "p50_ms_small_n": round(float(np.percentile(lat[small], 50)), 2) if small.any() else None,
                       "p99_ms_small_n": round(float(np.percentile(lat[small], 99)), 2) if small.any() else None,
                       "mean_batch": round(st["systems_done"] / max(st["batches"], 1), 2),
                       "failed": bad, "factor_gpops": round(
                           float(np.sum((2.0 if kind == "lu" else 1.0) * n.astype(np.float64) ** 3 / 3))
                           / span / 1e9, 1),
                       "same_requests": single},
            "roofline": None, "cpu_baseline": None,
        })
    return lines


def _serve_burst_vs_one_at_a_time(payload, n, nrhs, outs, args, dev, kind) -> dict:
    """The last rate's requests two more ways: all submitted at once to a new
    queue (its throughput with no arrival gaps), and one after another with
    the single-matrix calls (host -> device copy, getrf + getrs or potrf +
    potrs, copy back), the baseline the queue is compared with.  Every
    solution of both must equal the served one bit for bit."""
    import torch
    from paper_2401_14117_amd import posit32
    q = posit32.Queue(device_bytes=8 << 30, max_batch=1024, nb=args.nb, batch_max_n=args.batch_max_n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    req = posit32.REQ_LU if kind == "lu" else posit32.REQ_CHOL
    tickets = [q.submit(req, payload[int(k)][1][:, :int(r)], payload[int(k)][0])
               for k, r in zip(n, nrhs)]
    burst = [q.wait(t, 600.0) for t in tickets]
    burst_s = time.perf_counter() - t0
    q.close()
    same_burst = all(np.array_equal(b["X"], o["X"]) for b, o in zip(burst, outs))
    same = True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(len(n)):
        Ap, Bp = payload[int(n[i])]
        A = torch.from_numpy(Ap.view(np.int32)).to(dev)
        B = torch.from_numpy(np.ascontiguousarray(Bp[:, :int(nrhs[i])]).view(np.int32)).to(dev)
        if kind == "lu":
            _, ipiv, _ = posit32.getrf(A, args.nb)
            posit32.getrs(A, ipiv, B)
        else:
            posit32.potrf(A, args.nb)
            posit32.potrs(A, B)
        X = B.cpu().numpy().view(np.uint32)
        same = same and np.array_equal(X, outs[i]["X"])
    single_s = time.perf_counter() - t0
    return {"requests": int(len(n)),
            "queue_all_at_once": {"seconds": round(burst_s, 3), "solves_per_s": round(len(n) / burst_s, 1),
                                  "bit_identical_to_served": bool(same_burst)},
            "one_at_a_time": {"seconds": round(single_s, 3), "solves_per_s": round(len(n) / single_s, 1),
                              "bit_identical_to_served": bool(same)}}


def to_device_patterns(mat, dev):
    """FP64 values -> Posit(32,2) patterns with the library's own conversion;
    the sprinkled special values are then set by index."""
    import torch
    from paper_2401_14117_amd import posit32
    x = torch.from_numpy(np.ascontiguousarray(mat.values)).to(dev)
    p = posit32.from_f64(x)
    del x
    if mat.zero_mask is not None and mat.zero_mask.any():
        p[torch.from_numpy(mat.zero_mask).to(dev)] = 0
    if mat.nar_mask is not None and mat.nar_mask.any():
        p[torch.from_numpy(mat.nar_mask).to(dev)] = np.int32(-2 ** 31)
    return p


def run_cpu_baseline(case, budget_s: float):
    import oracle
    from paper_2401_14117_amd import workloads as W
    A = W.apply_masks(oracle.vec_from_double(case.A.values), case.A)
    B = W.apply_masks(oracle.vec_from_double(case.B.values), case.B)
    C = W.apply_masks(oracle.vec_from_double(case.C.values), case.C)
    al, be = oracle.from_double(case.alpha), oracle.from_double(case.beta)
    rng = np.random.default_rng(1234)
    threads = oracle.num_threads()
    # calibrate on a small sample, then size the sample to about budget_s
    count = max(threads, 16)
    t_cal = 0.0
    while True:
        rows = rng.integers(0, case.m, count)
        cols = rng.integers(0, case.n, count)
        t0 = time.perf_counter()
        oracle.gemm_entries(A, B, rows, cols, C[rows, cols], al, be)
        t_cal = time.perf_counter() - t0
        if t_cal > 0.5 or count >= case.m * case.n:
            break
        count *= 4
    per_entry = t_cal / count
    count = int(min(max(budget_s / per_entry, count), case.m * case.n))
    rows = rng.integers(0, case.m, count)
    cols = rng.integers(0, case.n, count)
    t0 = time.perf_counter()
    oracle.gemm_entries(A, B, rows, cols, C[rows, cols], al, be)
    dt = time.perf_counter() - t0
    gpops = 2.0 * count * case.k / dt / 1e9
    return {"value": round(gpops, 6), "unit": "Gpops/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} sampled C entries of {case.name} (each a full k={case.k} "
                      f"posit dot product plus alpha/beta epilogue), {dt:.1f} s on "
                      f"{threads} OpenMP threads"}


def _cpu_info() -> dict:
    """The GPU machine's host CPU: model, the cores this process may run on, and
    the OpenMP threads the oracle uses."""
    import oracle
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "affinity_cores": len(os.sched_getaffinity(0)),
            "omp_threads": oracle.num_threads()}


def run_cpu_single_thread(budget_s: float) -> dict:
    """The oracle on one thread at n = 1024 (square Rgemm case), sampled
    outputs for about budget_s seconds."""
    import ctypes
    import oracle
    from paper_2401_14117_amd import workloads as W
    oracle.lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    before = oracle.num_threads()
    gomp.omp_set_num_threads(1)
    try:
        r = run_cpu_baseline(W.gemm_square(1024), budget_s)
    finally:
        gomp.omp_set_num_threads(before)
    return {"value": r["value"], "unit": "Gpops/s", "threads": 1, "sample": r["sample"]}


def run_extras(args, dev) -> dict:
    """The other two clauses of the metric, measured in the same run: the
    20,000-system batched factor + solve (one launch, replayed
    from a hipGraph) for LU and Cholesky, and the LU request queue under
    Poisson arrivals at one rate with the same requests one at a time."""
    import argparse as _ap
    out = {}
    bargs = _ap.Namespace(**vars(args))
    bargs.cpu_budget = 0.0
    bargs.single_count = args.extras_single
    bargs.steps, bargs.warmup = 3, 1
    for kind in ("lu", "chol"):
        r = run_batch_bench(f"batch_{kind}", bargs, dev)
        c = r["config"]
        one = c["one_at_a_time"]
        out[f"batch_{kind}"] = {
            "solves_per_s": r["value"], "ms_per_batch": r["ms_per_step"], "systems": c["count"],
            "factor_gpops": c["factor_gpops"], "graph_bit_identical_to_eager": c["graph_bit_identical_to_eager"],
            "roofline_frac": (r["roofline"] or {}).get("frac"),
            "one_at_a_time_solves_per_s": one["solves_per_s"] if one else None,
            "one_at_a_time_bit_identical": one["bit_identical_to_batched"] if one else None,
            "setup_s": c["setup_s"]}
    sargs = _ap.Namespace(**vars(args))
    sargs.qps = [args.extras_qps]
    line = run_serve_bench(sargs, dev, "lu")[0]
    c = line["config"]
    same = c["same_requests"] or {}
    out["serve_lu"] = {
        "qps": c["qps"], "requests": c["requests"], "solves_per_s": line["value"],
        "p50_ms": c["p50_ms"], "p99_ms": c["p99_ms"], "p50_ms_small_n": c["p50_ms_small_n"],
        "p99_ms_small_n": c["p99_ms_small_n"], "mean_batch": c["mean_batch"], "failed": c["failed"],
        "all_at_once_solves_per_s": same.get("queue_all_at_once", {}).get("solves_per_s"),
        "one_at_a_time_solves_per_s": same.get("one_at_a_time", {}).get("solves_per_s"),
        "bit_identical": bool(same.get("queue_all_at_once", {}).get("bit_identical_to_served")
                              and same.get("one_at_a_time", {}).get("bit_identical_to_served"))}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="square_n8192",
                    help="square_nN | trailing_jJ | uniform_nN | normal_sigmaS_nN (Rgemm), "
                         "getrf_nN | potrf_nN (factor+solve), batch_lu | batch_chol (batched "
                         "factor+solve), serve_lu | serve_chol (request queue), ew_OP_IR | ew_all "
                         "(elementwise, OP in add/mul/div/sqrt, R in 0..4)")
    ap.add_argument("--trans", default="nn", choices=["nn", "nt", "tn", "tt"],
                    help="Rgemm transposes op(A), op(B) (square workloads reuse the buffers)")
    ap.add_argument("--ew-n", type=int, default=1 << 26, help="elements of the elementwise workloads")
    ap.add_argument("--batch-count", type=int, default=20000, help="systems of the batched workloads")
    ap.add_argument("--qps", type=float, nargs="+", default=[25.0, 50.0, 100.0, 150.0],
                    help="arrival rates of the serving workload (requests per second)")
    ap.add_argument("--power-seconds", type=float, default=8.0,
                    help="factor + solve workloads: seconds of repeated runs while GPU package power "
                         "is sampled with amd-smi (0: skip)")
    ap.add_argument("--batch-max-n", type=int, default=512,
                    help="serving workload: largest n the queue sends through the batched kernels")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of each arrival stream of the serving workload")
    ap.add_argument("--single-count", type=int, default=300,
                    help="sampled systems timed one at a time beside the batched workloads (0: skip)")
    ap.add_argument("--nb", type=int, default=256, help="block size of the factorisations")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0 = skip)")
    ap.add_argument("--extras", type=int, default=1,
                    help="Rgemm workloads: also measure the batched (LU, Cholesky) and served (LU) "
                         "workloads and the one-thread oracle, reported in the same line (0: skip)")
    ap.add_argument("--extras-qps", type=float, default=200.0,
                    help="arrival rate of the served workload measured with --extras")
    ap.add_argument("--extras-single", type=int, default=100,
                    help="batched systems also solved one at a time with --extras")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy (for HBM counter scaling) and exit")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU only; the multi-GPU Rgemm is a design "
              "(row blocks of C per GPU, one broadcast of B) and is not implemented",
              file=sys.stderr)
        return 2

    import torch
    from paper_2401_14117_amd import posit32
    posit32.lib()
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        x = torch.ones(256 << 20, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4}))
        return 0

    if args.workload.startswith(("getrf_n", "potrf_n")):
        print(json.dumps(run_solve_bench(args.workload, args, dev)))
        return 0
    if args.workload in ("serve_lu", "serve_chol"):
        for line in run_serve_bench(args, dev, args.workload[len("serve_"):]):
            print(json.dumps(line), flush=True)
        return 0
    if args.workload in ("batch_lu", "batch_chol"):
        print(json.dumps(run_batch_bench(args.workload, args, dev)))
        return 0
    if args.workload == "ew_all":                 # the whole Table 2 grid, one line each
        for r in ("I0", "I1", "I2", "I3", "I4"):
            for op in EW_OPS:
                print(json.dumps(run_elementwise_bench(f"ew_{op}_{r}", args, dev)), flush=True)
        return 0
    if args.workload.startswith("ew_"):
        print(json.dumps(run_elementwise_bench(args.workload, args, dev)))
        return 0

    case = make_case(args.workload)
    ta, tb = args.trans[0] == "t", args.trans[1] == "t"
    if (ta or tb) and not (case.m == case.n == case.k):
        raise SystemExit("--trans needs a square workload")
    t0 = time.perf_counter()
    A = to_device_patterns(case.A, dev)
    B = to_device_patterns(case.B, dev)
    C0 = to_device_patterns(case.C, dev)
    # alpha/beta patterns through the library conversion as well
    ab = posit32.from_f64(torch.tensor([case.alpha, case.beta], dtype=torch.float64, device=dev))
    alpha, beta = (int(v) & 0xFFFFFFFF for v in ab.cpu().tolist())
    C = torch.empty_like(C0)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    stream = torch.cuda.current_stream()

    def step(ev0=None, ev1=None):
        C.copy_(C0)
        if ev0 is not None:
            ev0.record(stream)
        posit32.gemm(A, B, C, alpha, beta, transa=ta, transb=tb)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in evs:
        step(e0, e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [e0.elapsed_time(e1) for e0, e1 in evs]

    m, n, k = case.m, case.n, case.k
    madds = m * n * k
    ms_per_step = wall * 1e3 / args.steps
    gpops = 2.0 * madds / (ms_per_step * 1e-3) / 1e9
    kavg = float(np.mean(kernel_ms))

    valu = load_valu_per_madd()
    roof = {"bound": "alu", "achieved": None, "peak": round(PEAK_INT_TOPS, 2),
            "unit": "Tlane-op/s", "frac": None, "traffic": load_traffic(args.workload) if args.trans == "nn" else None,
            "kernel_ms": round(kavg, 3), "valu_per_madd": valu,
            "kernel_gpops": round(2.0 * madds / (kavg * 1e-3) / 1e9, 2)}
    if valu is not None:
        achieved = valu * madds / (kavg * 1e-3) / 1e12
        roof["achieved"] = round(achieved, 3)
        roof["frac"] = round(achieved / PEAK_INT_TOPS, 4)

    cpu = None
    if args.cpu_budget > 0 and args.trans == "nn":
        cpu = run_cpu_baseline(case, args.cpu_budget)
        cpu.update(_cpu_info())
        cpu["single_thread_n1024"] = run_cpu_single_thread(min(args.cpu_budget, 5.0))
    extras = run_extras(args, dev) if args.extras and args.trans == "nn" and case.name == "square_n8192" else None

    out = {
        "metric": "Posit32 Rgemm Gpops/s at n=8192 (% int-VALU peak); batched solves/s; p50/p99 latency",
        "value": round(gpops, 2),
        "unit": "Gpops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "posit32 (int32 VALU)",
        "data": "synthetic",
        "config": {"workload": case.name, "m": m, "n": n, "k": k, "trans": args.trans,
                   "alpha": case.alpha, "beta": case.beta,
                   "inputs": "uniform[-1,1]*2^s, s in [-12,12], NaR/0 sprinkle 1e-6"
                   if "square" in case.name or "trailing" in case.name else
                   ("normal(0, sigma)" if "normal" in case.name else "uniform[-1,1]"),
                   "setup_s": round(setup_s, 2)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if extras is not None:
        out["batched"] = {k: v for k, v in extras.items() if k.startswith("batch_")}
        out["serving"] = extras["serve_lu"]
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
