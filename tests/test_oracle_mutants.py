"""Plausible mistakes planted in a copy of the oracle must fail the pins.

Each mutant is a one-line textual change to ``oracle/posit_oracle.c``,
compiled on the CPU into a throw-away library.  For each one, at least one
pinned fact (exact-checker results over all Posit(8,2) pairs, sampled
Posit(32,2) pairs, the fixed encodings, the accumulation-order and k-order
cases, the small-integer GEMM identity) must come out different.
"""
import ctypes
import functools
import os
import random
import subprocess
import tempfile

import numpy as np
import pytest

from tests import exact_checker as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "posit_oracle.c")

MUTANTS = {
    "tie_away_from_zero": ("if (G && (S || (P & 1u))) P += 1u;", "if (G) P += 1u;"),
    "sticky_off_by_one": ("S |= x_any_below(x, i0 + 1);", "S |= x_any_below(x, i0);"),
    "regime_zero_run": ("d.k = r0 ? m - 1 : -m;", "d.k = r0 ? m - 1 : -m + 1;"),
    "exponent_not_left_aligned": ("    e <<= 1;\n    if (i >= 0)", "    e <<= (i >= 0);\n    if (i >= 0)"),
    "no_saturation_at_maxpos": ("} else if (sc >= maxsc) {", "} else if (0) {"),
    "no_saturation_at_minpos": ("} else if (sc < -maxsc ||", "} else if (sc < -maxsc - 4 ||"),
    "product_sign": ("  x.neg = da.neg ^ db.neg;\n  unsigned __int128 prod", "  x.neg = da.neg;\n  unsigned __int128 prod"),
    "cancellation_sign": ("    r.neg = big->neg;", "    r.neg = a->neg;"),
    "sqrt_odd_exponent": ("if (ex & 1) { s <<= 1; ex -= 1; }", "if (ex & 1) { ex -= 1; }"),
    "gemm_descending_k": ("uint32_t a = transa ? A[p * lda + i] : A[i * lda + p];",
                          "uint32_t a = transa ? A[(k-1-p) * lda + i] : A[i * lda + (k-1-p)];"),
    "gemm_transb_ignored": ("uint32_t b = transb ? B[j * ldb + p] : B[p * ldb + j];",
                            "uint32_t b = B[p * ldb + j];"),
    "gemm_beta_first": ("  uint32_t acc = 0;\n  for (int64_t p = 0; p < k; ++p) {",
                        "  uint32_t acc = beta == 0 ? 0u : p32_mul(beta, cij); beta = 0;\n  for (int64_t p = 0; p < k; ++p) {"),
    "fraction_length": ("d.fs = i + 1 > 0 ? i + 1 : 0;", "d.fs = i > 0 ? i : 0;"),
}


def _build(src_text, d, name):
    path = os.path.join(d, name + ".c")
    with open(path, "w") as f:
        f.write(src_text)
    lib = os.path.join(d, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-I",
                           os.path.join(ROOT, "oracle"), "-o", lib, path, "-lm"])
    L = ctypes.CDLL(lib)
    L.oracle_vec_binop.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [ctypes.c_void_p] * 3
    L.oracle_vec_from_double.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    L.oracle_gemm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                              ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                              ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int64]
    return L


@functools.lru_cache(maxsize=None)
def _p8_expected():
    a = np.repeat(np.arange(256, dtype=np.uint32), 256)
    b = np.tile(np.arange(256, dtype=np.uint32), 256)
    exp = {
        0: np.array([X.add(8, int(x), int(y)) for x, y in zip(a, b)], dtype=np.uint32),
        2: np.array([X.mul(8, int(x), int(y)) for x, y in zip(a, b)], dtype=np.uint32),
        3: np.array([X.div(8, int(x), int(y)) for x, y in zip(a, b)], dtype=np.uint32),
        4: np.array([X.sqrt(8, int(x)) for x in a], dtype=np.uint32),
    }
    return a, b, exp


@functools.lru_cache(maxsize=None)
def _p32_probe():
    rng = random.Random(77)
    pats = []
    for _ in range(300):
        m = rng.randint(1, 31)
        lead = rng.randint(0, 1)
        body = str(lead) * m + (str(1 - lead) if m < 31 else "")
        while len(body) < 31:
            body += str(rng.randint(0, 1))
        p = int(body, 2)
        pats.append(((1 << 32) - p) & 0xFFFFFFFF if rng.randint(0, 1) else p)
    a = np.array(pats, dtype=np.uint32)
    b = np.array(pats[::-1], dtype=np.uint32)
    exp = {
        0: np.array([X.add(32, int(x), int(y)) for x, y in zip(a, b)], dtype=np.uint32),
        2: np.array([X.mul(32, int(x), int(y)) for x, y in zip(a, b)], dtype=np.uint32),
        4: np.array([X.sqrt(32, int(x)) for x in a], dtype=np.uint32),
    }
    return a, b, exp


def _caught(L):
    """Return the name of the first pin the library violates, or None."""
    a, b, exp = _p8_expected()
    out = np.empty_like(a)
    for op, e in exp.items():
        L.oracle_vec_binop(8, op, a.size, a.ctypes.data, b.ctypes.data, out.ctypes.data)
        if not np.array_equal(out, e):
            return f"p8 op {op}"
    a, b, exp = _p32_probe()
    out = np.empty_like(a)
    for op, e in exp.items():
        L.oracle_vec_binop(32, op, a.size, a.ctypes.data, b.ctypes.data, out.ctypes.data)
        if not np.array_equal(out, e):
            return f"p32 op {op}"
    # fixed encodings (1.0, maxpos, minpos, saturation beyond them)
    xs = np.array([1.0, 2.0 ** 120, 2.0 ** -120, 2.0 ** 130, 2.0 ** -130, -1.0], dtype=np.float64)
    want = np.array([0x40000000, 0x7FFFFFFF, 1, 0x7FFFFFFF, 1, 0xC0000000], dtype=np.uint32)
    got = np.empty(6, dtype=np.uint32)
    L.oracle_vec_from_double(32, 6, xs.ctypes.data, got.ctypes.data)
    if not np.array_equal(got, want):
        return "encodings"

    def gemm(A, B, C, ta=0, tb=0, m=None, n=None, k=None):
        A, B = np.ascontiguousarray(A), np.ascontiguousarray(B)
        C = np.array(C, dtype=np.uint32, copy=True)
        m = m if m is not None else C.shape[0]
        n = n if n is not None else C.shape[1]
        k = k if k is not None else (A.shape[0] if ta else A.shape[1])
        L.oracle_gemm(ta, tb, m, n, k, 0x40000000, A.ctypes.data, A.shape[1], B.ctypes.data,
                      B.shape[1], 0x40000000, C.ctypes.data, C.shape[1])
        return C

    def enc(x):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        out = np.empty(x.shape, dtype=np.uint32)
        L.oracle_vec_from_double(32, x.size, x.ctypes.data, out.ctypes.data)
        return out

    # order of accumulation: acc from 0, C added last
    if gemm(enc([[2.0 ** -28, 2.0 ** -28]]), enc([[1.0], [1.0]]), enc([[1.0]]))[0, 0] != 0x40000001:
        return "accumulation order"
    if gemm(enc([[2.0 ** 30, 1.0, -(2.0 ** 30)]]), enc([[1.0], [1.0], [1.0]]), enc([[0.0]]))[0, 0] != 0:
        return "ascending k"
    # small integers: exact, equal to integer matmul, with transposes
    rng = np.random.default_rng(1)
    A = rng.integers(-8, 8, (5, 6), endpoint=True)
    B = rng.integers(-8, 8, (4, 6), endpoint=True)
    C = rng.integers(-8, 8, (5, 4), endpoint=True)
    got = gemm(enc(A), enc(B), enc(C), tb=1, k=6)
    if not np.array_equal(got, enc(A @ B.T + C)):
        return "textbook transb"
    return None


def test_unmutated_oracle_passes():
    src = open(SRC).read()
    with tempfile.TemporaryDirectory() as d:
        assert _caught(_build(src, d, "orig")) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found for {name}"
    with tempfile.TemporaryDirectory() as d:
        L = _build(src.replace(old, new), d, name)
        assert _caught(L) is not None, f"mutant {name} survived the pins"
