"""Autotuner of the batched factorisations: the sub-panel width per size bucket.

The batched kernels (posit32_vbatched) factor every panel in
sub-panels of `sub` columns: inside a sub-panel the unblocked pivot search,
division and rank-1 updates; outside it fused-update chains on the Rgemm tile
routine; the solves work in blocks of 64 rows.  The width regroups the work
without changing the order in which any element receives its updates, so
every width gives the same bits -- it only moves time between the
latency-bound unblocked steps and the throughput-bound tiles, and the best
trade depends on the order n (a width of at least n factors a small matrix
unblocked, with no tile overhead).

tune() times every candidate width on synthetic systems of each size bucket
(the recipes of the batched workload: LU entries uniform[-1, 1], Cholesky
M M^T / n + I with M uniform[-1, 1], right-hand sides A * ones), checks that all
candidates produce identical factors, pivots, info and solutions, and keeps
the fastest width of each bucket.  write() stores the tables as
tuning/<arch>.json beside this module, where posit32.active_tuning() finds
them for VBatch and Queue.

    python -m paper_2401_14117_amd.autotune            # tune, write tuning/<arch>.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from paper_2401_14117_amd import posit32

# upper bounds of the size buckets (inclusive; the last one takes every larger n)
BUCKETS = (23, 47, 95, 191, 383, 2**31 - 1)
# the orders timed in each bucket (log-uniform between these bounds)
RANGES = ((16, 23), (24, 47), (48, 95), (96, 191), (192, 383), (384, 512))
# systems per bucket: enough work that each timing is well above launch noise
COUNTS = (6000, 4000, 2000, 800, 400, 200)
CANDIDATES = (8, 16, 24, 32, 48, 64)


class _BucketBatch:
    """count systems with n log-uniform in [lo, hi], resident on the device,
    with a pristine copy to restore before every timed run."""

    def __init__(self, kind: str, lo: int, hi: int, count: int, seed: int, dev):
        rng = np.random.default_rng(seed)
        ns = np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
        ns = np.sort(ns)[::-1]                      # decreasing n balances the workgroups
        nrhs = rng.integers(1, 16, size=count, endpoint=True).astype(np.int64)
        offa = np.concatenate([[0], np.cumsum(ns * ns)])
        offb = np.concatenate([[0], np.cumsum(ns * nrhs)])
        self.A0 = torch.empty(int(offa[-1]), dtype=torch.int32, device=dev)
        self.B0 = torch.empty(int(offb[-1]), dtype=torch.int32, device=dev)
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        for i, (n, r) in enumerate(zip(ns.tolist(), nrhs.tolist())):
            M = torch.rand((n, n), dtype=torch.float64, device=dev, generator=g) * 2.0 - 1.0
            if kind == "chol":
                A = M @ M.t().contiguous() / float(n) + torch.eye(n, dtype=torch.float64, device=dev)
            else:
                A = M
            B = A @ torch.ones((n, r), dtype=torch.float64, device=dev)
            posit32.from_f64(A, out=self.A0[int(offa[i]):int(offa[i + 1])])
            posit32.from_f64(B, out=self.B0[int(offb[i]):int(offb[i + 1])])
        self.A = self.A0.clone()
        self.B = self.B0.clone()
        As = [self.A[int(offa[i]):int(offa[i + 1])].view(int(ns[i]), int(ns[i])) for i in range(count)]
        Bs = [self.B[int(offb[i]):int(offb[i + 1])].view(int(ns[i]), int(nrhs[i])) for i in range(count)]
        self.vb = posit32.VBatch(As, Bs, lu=(kind == "lu"))
        self.ns = ns

    def run(self, tuning, nb: int) -> float:
        """Restore the inputs, factor and solve every system; kernel ms."""
        self.A.copy_(self.A0)
        self.B.copy_(self.B0)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        self.vb.run(True, True, nb, tuning=tuning)
        e1.record(s)
        e1.synchronize()
        return float(e0.elapsed_time(e1))

    def outputs(self):
        parts = [self.A.clone(), self.B.clone(), self.vb.info.clone()]
        if self.vb.ipivs is not None:
            parts += [p.clone() for p in self.vb.ipivs]
        return parts


def _uniform(width: int) -> posit32.Tuning:
    return posit32.Tuning.make([2**31 - 1], [width])


def tune(kinds=("lu", "chol"), buckets=BUCKETS, ranges=RANGES, counts=COUNTS, candidates=CANDIDATES,
         nb: int = 256, reps: int = 3, seed: int = 9000, log=print) -> dict:
    """Measure every candidate width in every bucket; returns the tables with
    the timings behind them."""
    if not (len(buckets) == len(ranges) == len(counts)) or len(buckets) > posit32.TUNE_BUCKETS:
        raise ValueError("one range and one count per bucket, at most 8 buckets")
    dev = torch.device("cuda", torch.cuda.current_device())
    props = torch.cuda.get_device_properties(dev)
    out = {"device": props.name, "arch": props.gcnArchName.split(":")[0],
           "compute_units": props.multi_processor_count, "nb": nb, "candidates": list(candidates),
           "recipe": {"ranges": [list(r) for r in ranges], "counts": list(counts), "seed": seed,
                      "reps": reps},
           "identical_results": True}
    t0 = time.perf_counter()
    for kind in kinds:
        subs, times = [], []
        for b, ((lo, hi), count) in enumerate(zip(ranges, counts)):
            batch = _BucketBatch(kind, lo, hi, count, seed + 100 * b + (0 if kind == "lu" else 50), dev)
            ref = None
            row = []
            for w in candidates:
                t = _uniform(w)
                batch.run(t, nb)                   # warm-up, and the result to compare
                got = batch.outputs()
                if ref is None:
                    ref = got
                elif not all(torch.equal(x, y) for x, y in zip(ref, got)):
                    out["identical_results"] = False
                    raise RuntimeError(f"{kind} bucket {b}: width {w} changed the results")
                row.append(min(batch.run(t, nb) for _ in range(reps)))
            best = candidates[int(np.argmin(row))]
            subs.append(best)
            times.append([round(x, 4) for x in row])
            log(f"{kind} n in [{lo}, {hi}] x{count}: " +
                "  ".join(f"{w}:{x:.3f}ms" for w, x in zip(candidates, row)) + f"  -> {best}")
            del batch
        out[kind] = {"max_n": list(buckets), "sub": subs, "ms": times}
    out["tuning_seconds"] = round(time.perf_counter() - t0, 1)
    return out


def default_path() -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return os.path.join(posit32.TUNING_DIR, f"{arch}.json")


def write(result: dict, path: str | None = None) -> str:
    path = path or default_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(result, f, indent=1)
        f.write("\n")
    return path


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=None, help="output JSON (default: tuning/<arch>.json)")
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--kinds", nargs="+", default=["lu", "chol"], choices=["lu", "chol"])
    args = ap.parse_args()
    res = tune(kinds=tuple(args.kinds), nb=args.nb, reps=args.reps)
    print("wrote", write(res, args.out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
