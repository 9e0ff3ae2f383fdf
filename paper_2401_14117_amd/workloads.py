"""Seeded synthetic workloads (FP64 values plus special-value masks).

This module only draws random numbers; it contains none of the posit
arithmetic.  Both the GPU path (through the library's own FP64 -> posit
conversion) and the CPU oracle (through its own conversion) consume what it
returns, so the two sides see the same inputs without sharing any code.

Workload recipes (all draws use ``numpy.random.default_rng(seed)`` in the order
listed, row-major):

* ``gemm_uniform``: A (m x k), B (k x n), C (m x n), each ``uniform(-1, 1)``.
  At m = n = k = 128, seed 1, this is the small Rgemm case.
* ``gemm_scaled``: each of A, B, C in turn draws U = uniform(-1, 1),
  S = integers(-12, 12, inclusive), X = U * 2^S, then M = random() < 1e-6 and
  Z = random() < 0.5; entries with M & Z become 0 and entries with M & ~Z
  become NaR after conversion.  Square sizes use seed 2000 + n with
  alpha = beta = 1; the trailing-update shapes m = n = 8192 - 256 j, k = 256
  use seed 3000 + j with alpha = -1, beta = 1.
* ``gemm_normal``: normal(0, sigma) entries, the paper's GEMM inputs
  (Section 4.3); used for the magnitude sweep, sigma in {1e-2, 1, 1e2, 1e4,
  1e6}, seed 77, alpha = beta = 1.
* ``elementwise_range``: the operand arrays p and q of the elementwise
  microbenchmark, each ``uniform(a, b)`` over one of the paper's magnitude
  ranges I0..I4 (Section 4.2, Table 2), seed 8000 + range index.  Values
  beyond maxpos or below minpos saturate on conversion, as they would in any
  posit program fed these inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Matrix:
    values: np.ndarray                      # float64, row-major
    zero_mask: np.ndarray | None = None     # entries forced to posit 0
    nar_mask: np.ndarray | None = None      # entries forced to NaR


@dataclass
class GemmCase:
    name: str
    m: int
    n: int
    k: int
    alpha: float
    beta: float
    A: Matrix
    B: Matrix
    C: Matrix
    meta: dict = field(default_factory=dict)


def _scaled(rng, shape, smin=-12, smax=12, sprinkle=1e-6) -> Matrix:
    u = rng.uniform(-1.0, 1.0, shape)
    s = rng.integers(smin, smax, size=shape, endpoint=True)
    x = np.ldexp(u, s.astype(np.int32))      # exact: scaling by a power of 2
    m = rng.random(shape) < sprinkle
    z = rng.random(shape) < 0.5
    return Matrix(x, m & z, m & ~z)


def gemm_uniform(m=128, n=128, k=128, seed=1) -> GemmCase:
    rng = np.random.default_rng(seed)
    A = Matrix(rng.uniform(-1.0, 1.0, (m, k)))
    B = Matrix(rng.uniform(-1.0, 1.0, (k, n)))
    C = Matrix(rng.uniform(-1.0, 1.0, (m, n)))
    return GemmCase(f"uniform_m{m}_n{n}_k{k}_seed{seed}", m, n, k, 1.0, 1.0, A, B, C)


def gemm_scaled(m, n, k, seed, alpha=1.0, beta=1.0, sprinkle=1e-6) -> GemmCase:
    rng = np.random.default_rng(seed)
    A = _scaled(rng, (m, k), sprinkle=sprinkle)
    B = _scaled(rng, (k, n), sprinkle=sprinkle)
    C = _scaled(rng, (m, n), sprinkle=sprinkle)
    return GemmCase(f"scaled_m{m}_n{n}_k{k}_seed{seed}", m, n, k, alpha, beta, A, B, C)


def gemm_square(n: int) -> GemmCase:
    """Square sweep case n in {1024, 2048, 4096, 8192}: seed 2000 + n."""
    c = gemm_scaled(n, n, n, 2000 + n)
    c.name = f"square_n{n}"
    return c


def gemm_trailing(j: int, N: int = 8192, kb: int = 256) -> GemmCase:
    """Trailing-update shape m = n = N - kb*j, k = kb: seed 3000 + j."""
    mn = N - kb * j
    c = gemm_scaled(mn, mn, kb, 3000 + j, alpha=-1.0, beta=1.0)
    c.name = f"trailing_j{j}_m{mn}_k{kb}"
    return c


def gemm_normal(n: int, sigma: float, seed: int = 77) -> GemmCase:
    rng = np.random.default_rng(seed)
    A = Matrix(rng.normal(0.0, sigma, (n, n)))
    B = Matrix(rng.normal(0.0, sigma, (n, n)))
    C = Matrix(rng.normal(0.0, sigma, (n, n)))
    return GemmCase(f"normal_n{n}_sigma{sigma:g}", n, n, n, 1.0, 1.0, A, B, C)


def apply_masks(patterns: np.ndarray, mat: Matrix) -> np.ndarray:
    """Set the sprinkled special values on an array of posit32 patterns."""
    if mat.zero_mask is not None:
        patterns[mat.zero_mask] = 0
    if mat.nar_mask is not None:
        patterns[mat.nar_mask] = 0x80000000
    return patterns


@dataclass
class SolveCase:
    name: str
    n: int
    A: np.ndarray          # float64 n x n
    b: np.ndarray          # float64 n x nrhs
    kind: str              # "lu" or "chol"


def lu_case(n: int, nrhs: int = 1) -> SolveCase:
    """LU factor+solve input: A ~ uniform[-1,1] (seed 4000+n), b = A * ones."""
    rng = np.random.default_rng(4000 + n)
    A = rng.uniform(-1.0, 1.0, (n, n))
    b = A @ np.ones((n, nrhs))
    return SolveCase(f"getrf_n{n}", n, A, b, "lu")


def chol_case(n: int, nrhs: int = 1) -> SolveCase:
    """Cholesky factor+solve input: A = B B^T / n + I with B ~ uniform[-1,1]
    (seed 5000+n), b = A * ones."""
    rng = np.random.default_rng(5000 + n)
    Bm = rng.uniform(-1.0, 1.0, (n, n))
    A = Bm @ Bm.T / n + np.eye(n)
    b = A @ np.ones((n, nrhs))
    return SolveCase(f"potrf_n{n}", n, A, b, "chol")


# magnitude ranges [a, b) of the paper's elementwise kernel study (Table 2)
RANGES = {
    "I0": (1.0, 2.0),
    "I1": (1e-38, 1e-30),
    "I2": (1e30, 1e38),
    "I3": (1e-15, 1e-14),
    "I4": (1e14, 1e15),
}


def elementwise_range(n: int, rng_name: str) -> tuple[np.ndarray, np.ndarray]:
    """p, q ~ uniform[a, b) for range rng_name (seed 8000 + its index)."""
    a, b = RANGES[rng_name]
    rng = np.random.default_rng(8000 + int(rng_name[1:]))
    p = rng.uniform(a, b, n)
    q = rng.uniform(a, b, n)
    return p, q


@dataclass
class BatchCase:
    name: str
    kind: str                 # "lu" or "chol"
    n: np.ndarray             # int64 [count]
    nrhs: np.ndarray          # int64 [count]
    seed: int


def batch_sizes(count: int = 20000, seed: int = 6000) -> tuple[np.ndarray, np.ndarray]:
    """Sizes of the batched workload: n = round(exp(U(ln 16, ln 512))) and
    nrhs = integers(1, 16, inclusive), drawn in that order."""
    rng = np.random.default_rng(seed)
    n = np.round(np.exp(rng.uniform(np.log(16), np.log(512), count))).astype(np.int64)
    nrhs = rng.integers(1, 16, size=count, endpoint=True).astype(np.int64)
    return n, nrhs


def batch_matrices(kind: str, n: np.ndarray, nrhs: np.ndarray, seed: int = 6000, start: int = 0,
                   stop: int | None = None):
    """Yield (i, A, B) for systems start..stop-1 of the batched workload.  System
    i draws from its own generator seeded (seed, i): LU entries uniform[-1, 1];
    Cholesky A = M M^T / n + I with M uniform[-1, 1]; B = A * ones(n, nrhs)."""
    stop = len(n) if stop is None else stop
    for i in range(start, stop):
        rng = np.random.default_rng([seed, i])
        k = int(n[i])
        M = rng.uniform(-1.0, 1.0, (k, k))
        A = M if kind == "lu" else M @ M.T / k + np.eye(k)
        B = A @ np.ones((k, int(nrhs[i])))
        yield i, A, B


def serve_stream(qps: float, duration_s: float, seed: int = 7000):
    """Request stream of the serving workload: Poisson arrivals at rate qps
    over duration_s (exponential gaps), each request n = round(exp(U(ln 32,
    ln 2048))) and nrhs = integers(1, 32, inclusive).  Returns (arrival times,
    n, nrhs)."""
    rng = np.random.default_rng([seed, int(round(qps * 1000))])
    count = max(1, int(rng.poisson(qps * duration_s)))
    t = np.cumsum(rng.exponential(1.0 / qps, count))
    n = np.round(np.exp(rng.uniform(np.log(32), np.log(2048), count))).astype(np.int64)
    nrhs = rng.integers(1, 32, size=count, endpoint=True).astype(np.int64)
    return t, n, nrhs


def serve_system(n: int, nrhs: int, seed: int, kind: str = "lu"):
    """Payload of one served request (FP64): LU entries uniform[-1, 1],
    Cholesky M M^T / n + I; B uniform[-1, 1]; generator (seed, n, nrhs)."""
    rng = np.random.default_rng([seed, n, nrhs])
    M = rng.uniform(-1.0, 1.0, (n, n))
    A = M if kind == "lu" else M @ M.T / n + np.eye(n)
    B = rng.uniform(-1.0, 1.0, (n, nrhs))
    return A, B
