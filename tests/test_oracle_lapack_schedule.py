"""Pin of the oracle's factorisation schedule (the order of every rounded
operation of Rgetrf/Rgetrs and Rpotrf/Rpotrs, not only their invariants).

The paper factors with LAPACK's right-looking blocked algorithms and
accelerates only the trailing update with Rgemm (Section 3, Section 5.2); the
block size and the unblocked order are this library's reading, stated in
``oracle/ref_lapack.c``.  Here that reading is evaluated a second time, on tiny
systems (n <= 7, several block sizes), with the exact checker's arithmetic
(``tests/exact_checker.py``: exact rationals and a different rounding
algorithm) and in a different loop organisation where the reading allows one:

* the LU panel left-looking (column c first receives the updates of the
  panel's earlier columns, then its pivot search), which gives every element
  the same sequence of operations as the right-looking order of the reading;
* pivots chosen by comparing exact magnitudes (not pattern keys);
* U12 and both triangular solves element by element (each entry takes its
  updates in the stated order, from already final entries);
* the trailing updates through the checker's own Rgemm element (dot product
  from zero in ascending k, then alpha = -1 and beta = 1).

The transposed solve (A^T X = B from P A = L U) and the upper Cholesky
forms (A = U^T U) are evaluated the same way: the transposed solve element by
element with the interchanges applied as one permutation, the upper
factorisation in LAPACK's upper loop organisation (rows of U, not the
transposed lower factor the oracle takes), with the strict lower triangle
filled with patterns that must be neither read nor changed.

Factors, pivots, info and solutions must agree bit for bit.  Planted mistakes
in a copy of ``ref_lapack.c`` (an unblocked trailing update, a reciprocal in
place of the division, U12 in descending order, a missing division in
potrs, ties to the largest row) must each fail this comparison.
"""
import ctypes
import functools
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from tests import exact_checker as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N = 32
NAR = 0x80000000
ONE = 0x40000000
MINUS_ONE = 0xC0000000


# ---- the schedule, evaluated with the exact checker ---------------------------

def _neg(a):
    v = X.decode(N, a)
    return NAR if v is None else X.round_exact(N, -v)


def _fms(a, b, c):
    """a - rnd(b * c), every step rounded."""
    return X.add(N, a, _neg(X.mul(N, b, c)))


def _mag(a):
    """Magnitude for the pivot search: NaR below every number."""
    v = X.decode(N, a)
    return Fraction(-1) if v is None else abs(v)


def sched_getrf(A0, nb):
    A = [[int(x) for x in row] for row in A0]
    n = len(A)
    ipiv = list(range(n))
    info = 0
    for j in range(0, n, nb):
        je = min(j + nb, n)
        for c in range(j, je):
            # left-looking: column c (rows c..n-1) takes the updates of the
            # panel's earlier columns, in their order
            for cp in range(j, c):
                for i in range(cp + 1, n):
                    A[i][c] = _fms(A[i][c], A[i][cp], A[cp][c])
            p = c
            for i in range(c + 1, n):
                if _mag(A[i][c]) > _mag(A[p][c]):
                    p = i
            ipiv[c] = p
            if p != c:
                for q in range(j, je):
                    A[c][q], A[p][q] = A[p][q], A[c][q]
            piv = A[c][c]
            if piv == 0:
                info = info or c + 1
            else:
                for i in range(c + 1, n):
                    A[i][c] = X.div(N, A[i][c], piv)
        for c in range(j, je):
            p = ipiv[c]
            if p != c:
                for q in list(range(0, j)) + list(range(je, n)):
                    A[c][q], A[p][q] = A[p][q], A[c][q]
        # U12 entry by entry: row r of the block takes rows j..r-1 in order
        for r in range(j, je):
            for q in range(je, n):
                x = A[r][q]
                for c in range(j, r):
                    x = _fms(x, A[r][c], A[c][q])
                A[r][q] = x
        for i in range(je, n):
            for q in range(je, n):
                A[i][q] = X.gemm_element([A[i][p] for p in range(j, je)],
                                         [A[p][q] for p in range(j, je)], A[i][q], MINUS_ONE, ONE)
    return A, ipiv, info


def sched_getrs(LU, ipiv, B0):
    n, nrhs = len(B0), len(B0[0]) if len(B0) else 0
    B = [[int(x) for x in row] for row in B0]
    for c in range(n):
        B[c], B[ipiv[c]] = B[ipiv[c]], B[c]
    Y = [[0] * nrhs for _ in range(n)]
    for r in range(n):
        for q in range(nrhs):
            x = B[r][q]
            for c in range(r):
                x = _fms(x, LU[r][c], Y[c][q])
            Y[r][q] = x
    Xs = [[0] * nrhs for _ in range(n)]
    for r in range(n - 1, -1, -1):
        for q in range(nrhs):
            x = Y[r][q]
            for c in range(n - 1, r, -1):
                x = _fms(x, LU[r][c], Xs[c][q])
            Xs[r][q] = X.div(N, x, LU[r][r])
    return Xs


def sched_potrf(A0, nb):
    A = [[int(x) for x in row] for row in A0]
    n = len(A)
    for j in range(0, n, nb):
        je = min(j + nb, n)
        for c in range(j, je):
            v = X.decode(N, A[c][c])
            if v is None or v <= 0:
                return A, c + 1
            d = X.sqrt(N, A[c][c])
            A[c][c] = d
            for i in range(c + 1, je):
                A[i][c] = X.div(N, A[i][c], d)
            for i in range(c + 1, je):
                for q in range(c + 1, i + 1):
                    A[i][q] = _fms(A[i][q], A[i][c], A[q][c])
        for r in range(je, n):
            for c in range(j, je):
                x = A[r][c]
                for q in range(j, c):
                    x = _fms(x, A[r][q], A[c][q])
                A[r][c] = X.div(N, x, A[c][c])
        for i in range(je, n):
            for q in range(je, i + 1):
                A[i][q] = X.gemm_element([A[i][p] for p in range(j, je)],
                                         [A[q][p] for p in range(j, je)], A[i][q], MINUS_ONE, ONE)
    return A, 0


def sched_potrs(L, B0):
    n, nrhs = len(B0), len(B0[0]) if len(B0) else 0
    Y = [[0] * nrhs for _ in range(n)]
    for r in range(n):
        for q in range(nrhs):
            x = int(B0[r][q])
            for c in range(r):
                x = _fms(x, L[r][c], Y[c][q])
            Y[r][q] = X.div(N, x, L[r][r])
    Xs = [[0] * nrhs for _ in range(n)]
    for r in range(n - 1, -1, -1):
        for q in range(nrhs):
            x = Y[r][q]
            for c in range(n - 1, r, -1):
                x = _fms(x, L[c][r], Xs[c][q])
            Xs[r][q] = X.div(N, x, L[r][r])
    return Xs


def _perm_from_ipiv(ipiv):
    """Row i of P A is row perm[i] of A (the interchanges applied in order)."""
    perm = list(range(len(ipiv)))
    for c, p in enumerate(ipiv):
        perm[c], perm[p] = perm[p], perm[c]
    return perm


def sched_getrs_trans(LU, ipiv, B0):
    """A^T X = B with P A = L U: U^T Y = B, L^T Z = Y, X = P^T Z."""
    n, nrhs = len(B0), len(B0[0]) if len(B0) else 0
    Y = [[0] * nrhs for _ in range(n)]
    for r in range(n):
        for q in range(nrhs):
            x = int(B0[r][q])
            for c in range(r):
                x = _fms(x, LU[c][r], Y[c][q])
            Y[r][q] = X.div(N, x, LU[r][r])
    Z = [[0] * nrhs for _ in range(n)]
    for r in range(n - 1, -1, -1):
        for q in range(nrhs):
            x = Y[r][q]
            for c in range(n - 1, r, -1):
                x = _fms(x, LU[c][r], Z[c][q])
            Z[r][q] = x
    perm = _perm_from_ipiv(ipiv)
    Xs = [None] * n
    for i in range(n):
        Xs[perm[i]] = Z[i]
    return Xs


def sched_potrf_upper(A0, nb):
    """A = U^T U in LAPACK's upper organisation: row c of the diagonal block
    is divided by its root and updates the rows below it; then U12 column by
    column and the upper triangle of the trailing matrix by Rgemm elements
    (U12^T U12)."""
    A = [[int(x) for x in row] for row in A0]
    n = len(A)
    for j in range(0, n, nb):
        je = min(j + nb, n)
        for c in range(j, je):
            v = X.decode(N, A[c][c])
            if v is None or v <= 0:
                return A, c + 1
            d = X.sqrt(N, A[c][c])
            A[c][c] = d
            for q in range(c + 1, je):
                A[c][q] = X.div(N, A[c][q], d)
            for i in range(c + 1, je):
                for q in range(i, je):
                    A[i][q] = _fms(A[i][q], A[c][i], A[c][q])
        for r in range(je, n):
            for c in range(j, je):
                x = A[c][r]
                for q in range(j, c):
                    x = _fms(x, A[q][r], A[q][c])
                A[c][r] = X.div(N, x, A[c][c])
        for i in range(je, n):
            for q in range(i, n):
                A[i][q] = X.gemm_element([A[p][i] for p in range(j, je)],
                                         [A[p][q] for p in range(j, je)], A[i][q], MINUS_ONE, ONE)
    return A, 0


def sched_potrs_upper(U, B0):
    n, nrhs = len(B0), len(B0[0]) if len(B0) else 0
    Y = [[0] * nrhs for _ in range(n)]
    for r in range(n):
        for q in range(nrhs):
            x = int(B0[r][q])
            for c in range(r):
                x = _fms(x, U[c][r], Y[c][q])
            Y[r][q] = X.div(N, x, U[r][r])
    Xs = [[0] * nrhs for _ in range(n)]
    for r in range(n - 1, -1, -1):
        for q in range(nrhs):
            x = Y[r][q]
            for c in range(n - 1, r, -1):
                x = _fms(x, U[r][c], Xs[c][q])
            Xs[r][q] = X.div(N, x, U[r][r])
    return Xs


# ---- tiny cases ------------------------------------------------------------------

def _enc(x):
    """Posit(32,2) pattern of a binary64 value, rounded by the checker."""
    return X.round_exact(N, Fraction(float(x)))


def _regime_pattern(rng):
    m = int(rng.integers(1, 32))
    lead = int(rng.integers(0, 2))
    body = str(lead) * m + (str(1 - lead) if m < 31 else "")
    while len(body) < 31:
        body += str(int(rng.integers(0, 2)))
    p = int(body, 2)
    return ((1 << 32) - p) & 0xFFFFFFFF if rng.integers(0, 2) else p


def _matrix(kind, n, ncols, rng):
    if kind == "scaled":        # uniform[-1,1] * 2^s, the benchmark's recipe
        vals = rng.uniform(-1, 1, (n, ncols)) * 2.0 ** rng.integers(-12, 13, (n, ncols))
        return [[_enc(v) for v in row] for row in vals]
    if kind == "ties":          # small integers: equal magnitudes, exact sums
        vals = rng.integers(-2, 3, (n, ncols)).astype(float)
        return [[_enc(v) for v in row] for row in vals]
    if kind == "regimes":       # operands from every regime, with a zero and a NaR
        M = [[_regime_pattern(rng) for _ in range(ncols)] for _ in range(n)]
        if n * ncols >= 4:
            M[int(rng.integers(0, n))][int(rng.integers(0, ncols))] = 0
            M[int(rng.integers(0, n))][int(rng.integers(0, ncols))] = NAR
        return M
    if kind == "zero_pivot":    # uniform with a zero column (info) and a NaR
        vals = rng.uniform(-1, 1, (n, ncols))
        M = [[_enc(v) for v in row] for row in vals]
        zc = int(rng.integers(0, ncols))
        for i in range(n):
            M[i][zc] = 0
        if n > 2:
            M[n - 1][(zc + 1) % ncols] = NAR
        if n > 1 and rng.integers(0, 2):
            M[int(rng.integers(0, n))][zc] = NAR     # below a zero pivot: 0 stays the pivot
        return M
    raise ValueError(kind)


def _spd(kind, n, rng):
    if kind == "spd":           # B B^T / n + I from the benchmark's entries
        B = rng.uniform(-1, 1, (n, n)) * 2.0 ** rng.integers(-3, 4, (n, n))
        A = B @ B.T / n + np.eye(n)
        return [[_enc(v) for v in row] for row in A]
    if kind == "indefinite":    # fails at some column inside or after a block
        B = rng.uniform(-1, 1, (n, n))
        A = B @ B.T / n + np.eye(n) * 0.05
        A[n - 1 - int(rng.integers(0, min(n, 3))), n - 1 - int(rng.integers(0, min(n, 3)))] -= 3.0
        A = (A + A.T) / 2
        return [[_enc(v) for v in row] for row in A]
    if kind == "regimes":       # symmetric, positive diagonal, every regime
        M = [[0] * n for _ in range(n)]
        for i in range(n):
            for q in range(i + 1):
                p = _regime_pattern(rng)
                if i == q and p >= NAR:
                    p = ONE if p == NAR else ((1 << 32) - p) & 0xFFFFFFFF
                M[i][q] = M[q][i] = p
        return M
    raise ValueError(kind)


def _cases():
    out = []
    seed = 0
    for n in (1, 2, 3, 4, 5, 6, 7):
        for nb in sorted({1, 2, 3, n}):
            for kind in ("scaled", "ties", "regimes", "zero_pivot"):
                if kind == "zero_pivot" and n < 2:
                    continue
                out.append((n, nb, kind, seed))
                seed += 1
    return out


CASES = _cases()


def _chol_cases():
    out = []
    seed = 1000
    for n in (1, 2, 3, 4, 5, 6, 7):
        for nb in sorted({1, 2, 3, n}):
            for kind in ("spd", "indefinite", "regimes"):
                out.append((n, nb, kind, seed))
                seed += 1
    return out


CHOL_CASES = _chol_cases()


@functools.lru_cache(maxsize=None)
def _lu_expected(case):
    n, nb, kind, seed = case
    rng = np.random.default_rng(seed)
    A = _matrix(kind, n, n, rng)
    nrhs = 1 + seed % 3
    B = _matrix("scaled", n, nrhs, rng)
    LU, ipiv, info = sched_getrf(A, nb)
    Xs = sched_getrs(LU, ipiv, B)
    return (np.array(A, np.uint32), np.array(B, np.uint32).reshape(n, nrhs),
            np.array(LU, np.uint32), np.array(ipiv, np.int32), info,
            np.array(Xs, np.uint32).reshape(n, nrhs))


@functools.lru_cache(maxsize=None)
def _chol_expected(case):
    n, nb, kind, seed = case
    rng = np.random.default_rng(seed)
    A = _spd(kind, n, rng)
    nrhs = 1 + seed % 3
    B = _matrix("scaled", n, nrhs, rng)
    L, info = sched_potrf(A, nb)
    Xs = sched_potrs(L, B) if info == 0 else None
    return (np.array(A, np.uint32), np.array(B, np.uint32).reshape(n, nrhs), np.array(L, np.uint32),
            info, None if Xs is None else np.array(Xs, np.uint32).reshape(n, nrhs))


@functools.lru_cache(maxsize=None)
def _lu_trans_expected(case):
    A, B, LU, ipiv, info, _ = _lu_expected(case)
    Xs = sched_getrs_trans(LU.tolist(), ipiv.tolist(), B.tolist())
    return np.array(Xs, np.uint32).reshape(B.shape)


@functools.lru_cache(maxsize=None)
def _chol_upper_expected(case):
    """The lower case's symmetric matrix with its strict lower triangle
    replaced by unrelated patterns (never read by the upper form)."""
    n, nb, kind, seed = case
    A, B, _, _, _ = _chol_expected(case)
    rng = np.random.default_rng(seed + 50000)
    Au = A.copy()
    for i in range(n):
        for q in range(i):
            Au[i, q] = _regime_pattern(rng)
    U, info = sched_potrf_upper(Au.tolist(), nb)
    Xs = sched_potrs_upper(U, B.tolist()) if info == 0 else None
    return Au, np.array(U, np.uint32), info, None if Xs is None else np.array(Xs, np.uint32).reshape(B.shape)


# ---- the oracle (or a planted copy of it) on the same cases ------------------------

class _Lib:
    """The oracle's factorisation routines from a given shared library."""

    def __init__(self, L):
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.oracle_getrf.argtypes = [i64, i64, vp, i64, vp, vp]
        L.oracle_getrs.argtypes = [i64, i64, vp, i64, vp, vp, i64]
        L.oracle_potrf.argtypes = [i64, i64, vp, i64, vp]
        L.oracle_potrs.argtypes = [i64, i64, vp, i64, vp, i64]
        L.oracle_getrs_trans.argtypes = [i64, i64, vp, i64, vp, vp, i64]
        L.oracle_potrf_upper.argtypes = [i64, i64, vp, i64, vp]
        L.oracle_potrf_upper.restype = ctypes.c_int
        L.oracle_potrs_upper.argtypes = [i64, i64, vp, i64, vp, i64]
        self.L = L

    def getrf(self, A, nb):
        A = np.array(A, np.uint32, copy=True, order="C")
        n = A.shape[0]
        ipiv = np.zeros(n, np.int32)
        info = np.zeros(1, np.int32)
        self.L.oracle_getrf(n, nb, A.ctypes.data, n, ipiv.ctypes.data, info.ctypes.data)
        return A, ipiv, int(info[0])

    def getrs(self, LU, ipiv, B, trans=False):
        Bc = np.array(B, np.uint32, copy=True, order="C")
        LU = np.ascontiguousarray(LU, np.uint32)
        ipiv = np.ascontiguousarray(ipiv, np.int32)
        f = self.L.oracle_getrs_trans if trans else self.L.oracle_getrs
        f(LU.shape[0], Bc.shape[1], LU.ctypes.data, LU.shape[0], ipiv.ctypes.data, Bc.ctypes.data,
          Bc.shape[1])
        return Bc

    def potrf(self, A, nb, upper=False):
        A = np.array(A, np.uint32, copy=True, order="C")
        info = np.zeros(1, np.int32)
        if upper:
            assert self.L.oracle_potrf_upper(A.shape[0], nb, A.ctypes.data, A.shape[0], info.ctypes.data) == 0
        else:
            self.L.oracle_potrf(A.shape[0], nb, A.ctypes.data, A.shape[0], info.ctypes.data)
        return A, int(info[0])

    def potrs(self, L, B, upper=False):
        Bc = np.array(B, np.uint32, copy=True, order="C")
        L = np.ascontiguousarray(L, np.uint32)
        f = self.L.oracle_potrs_upper if upper else self.L.oracle_potrs
        f(L.shape[0], Bc.shape[1], L.ctypes.data, L.shape[0], Bc.ctypes.data, Bc.shape[1])
        return Bc


def _lu_mismatch(lib, case):
    A, B, LU, ipiv, info, Xs = _lu_expected(case)
    gLU, gipiv, ginfo = lib.getrf(A, case[1])
    if ginfo != info:
        return f"info {ginfo} != {info}"
    if not np.array_equal(gipiv, ipiv):
        return f"pivots {gipiv.tolist()} != {ipiv.tolist()}"
    if not np.array_equal(gLU, LU):
        return "factors differ"
    if not np.array_equal(lib.getrs(LU, ipiv, B), Xs):
        return "solution differs"
    if not np.array_equal(lib.getrs(LU, ipiv, B, trans=True), _lu_trans_expected(case)):
        return "transposed solution differs"
    return None


def _chol_mismatch(lib, case):
    A, B, L, info, Xs = _chol_expected(case)
    gL, ginfo = lib.potrf(A, case[1])
    if ginfo != info:
        return f"info {ginfo} != {info}"
    if not np.array_equal(gL, L):
        return "factor differs"
    if Xs is not None and not np.array_equal(lib.potrs(L, B), Xs):
        return "solution differs"
    Au, U, uinfo, UXs = _chol_upper_expected(case)
    gU, ginfo = lib.potrf(Au, case[1], upper=True)
    if ginfo != uinfo:
        return f"upper info {ginfo} != {uinfo}"
    if not np.array_equal(gU, U):
        return "upper factor differs"
    if UXs is not None and not np.array_equal(lib.potrs(U, B, upper=True), UXs):
        return "upper solution differs"
    return None


@functools.lru_cache(maxsize=None)
def _oracle():
    return _Lib(O.lib())


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}-nb{c[1]}-{c[2]}" for c in CASES])
def test_getrf_getrs_schedule(case):
    assert _lu_mismatch(_oracle(), case) is None


@pytest.mark.parametrize("case", CHOL_CASES, ids=[f"n{c[0]}-nb{c[1]}-{c[2]}" for c in CHOL_CASES])
def test_potrf_potrs_schedule(case):
    assert _chol_mismatch(_oracle(), case) is None


def test_cases_reach_the_rare_paths():
    """The tiny cases include zero pivots, NaR factors, failed Cholesky
    diagonals at several positions, pivot ties and row interchanges."""
    infos = [_lu_expected(c)[4] for c in CASES]
    assert sum(i > 0 for i in infos) >= 10
    assert any(np.any(_lu_expected(c)[2] == NAR) for c in CASES)
    assert sum(np.any(_lu_expected(c)[3] != np.arange(c[0])) for c in CASES) >= 30
    chol = [_chol_expected(c)[3] for c in CHOL_CASES]
    assert sum(i > 0 for i in chol) >= 10 and sum(i == 0 for i in chol) >= 20
    assert len({i for i in chol if i > 0}) >= 4
    # the upper form sees the same symmetric matrix: same info as the lower one
    assert [_chol_upper_expected(c)[2] for c in CHOL_CASES] == chol


# ---- planted mistakes in ref_lapack.c ----------------------------------------------

REF = os.path.join(ROOT, "oracle", "ref_lapack.c")

MUTANTS = {
    # the trailing update as unblocked rank-1 updates instead of Rgemm
    "unblocked_trailing_update": (
        """      oracle_gemm(0, 0, mm, mm, jb, MINUS_ONE, &A[(j + jb) * lda + j], lda,
                  &A[j * lda + j + jb], lda, ONE, &A[(j + jb) * lda + j + jb], lda);""",
        """      for (int64_t p = j; p < j + jb; ++p)
        for (int64_t i = j + jb; i < j + jb + mm; ++i)
          for (int64_t q = j + jb; q < n; ++q)
            A[i * lda + q] = pfms(A[i * lda + q], A[i * lda + p], A[p * lda + q]);"""),
    # multiplication by the pivot's reciprocal instead of the division
    "reciprocal_of_pivot": (
        "A[i * lda + c] = pdiv(A[i * lda + c], piv);",
        "A[i * lda + c] = pmul(A[i * lda + c], pdiv(ONE, piv));"),
    # U12 with the panel's columns in descending order
    "descending_u12": (
        "        for (int64_t c = j; c < j + jb; ++c)\n          for (int64_t r = c + 1; r < j + jb; ++r)",
        "        for (int64_t c = j + jb - 1; c >= j; --c)\n          for (int64_t r = c + 1; r < j + jb; ++r)"),
    # potrs's forward substitution without its division by L[c][c]
    "potrs_first_division_missing": (
        """  for (int64_t c = 0; c < n; ++c) {
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], L[c * lda + c]);""",
        """  for (int64_t c = 0; c < n; ++c) {"""),
    # ties of the pivot search to the largest row
    "pivot_ties_to_largest_row": ("if (key > best) { best = key; p = i; }",
                                  "if (key >= best) { best = key; p = i; }"),
    # the Cholesky trailing update as unblocked rank-1 updates
    "chol_unblocked_trailing_update": (
        """          uint32_t acc = 0;
          for (int64_t p = j; p < j + jb; ++p)
            acc = padd(acc, pmul(A[i * lda + p], A[q * lda + p]));
          const uint32_t r = pmul(MINUS_ONE, acc);
          A[i * lda + q] = padd(r, pmul(ONE, A[i * lda + q]));""",
        """          for (int64_t p = j; p < j + jb; ++p)
            A[i * lda + q] = pfms(A[i * lda + q], A[i * lda + p], A[q * lda + p]);"""),
    # L21's division taken before its updates
    "l21_division_first": (
        """          uint32_t x = A[r * lda + c];
          for (int64_t q = j; q < c; ++q) x = pfms(x, A[r * lda + q], A[c * lda + q]);
          A[r * lda + c] = pdiv(x, A[c * lda + c]);""",
        """          uint32_t x = pdiv(A[r * lda + c], A[c * lda + c]);
          for (int64_t q = j; q < c; ++q) x = pfms(x, pdiv(A[r * lda + q], A[c * lda + c]), A[c * lda + q]);
          A[r * lda + c] = x;"""),
    # getrs's backward substitution with the division after the updates of the rows above
    "getrs_backward_order": (
        """    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], LU[c * lda + c]);
    for (int64_t r = 0; r < c; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], LU[r * lda + c], B[c * ldb + q]);""",
        """    for (int64_t r = 0; r < c; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], pdiv(LU[r * lda + c], LU[c * lda + c]), B[c * ldb + q]);
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], LU[c * lda + c]);"""),
    # the transposed solve's interchanges applied in forward order
    "getrs_trans_pivots_forward": (
        """  for (int64_t c = n - 1; c >= 0; --c)
    if (ipiv[c] != c) swap_rows(B, ldb, c, ipiv[c], 0, nrhs);""",
        """  for (int64_t c = 0; c < n; ++c)
    if (ipiv[c] != c) swap_rows(B, ldb, c, ipiv[c], 0, nrhs);"""),
    # the transposed solve's backward step with L instead of L^T
    "getrs_trans_untransposed_l": (
        """        B[r * ldb + q] = pfms(B[r * ldb + q], LU[c * lda + r], B[c * ldb + q]);
  for (int64_t c = n - 1; c >= 0; --c)
    if (ipiv[c] != c)""",
        """        B[r * ldb + q] = pfms(B[r * ldb + q], LU[r * lda + c], B[c * ldb + q]);
  for (int64_t c = n - 1; c >= 0; --c)
    if (ipiv[c] != c)"""),
    # the upper Cholesky reading the lower triangle
    "potrf_upper_reads_lower": (
        "T[i * n + j] = j <= i ? A[j * lda + i] : 0u;",
        "T[i * n + j] = j <= i ? A[i * lda + j] : 0u;"),
    # the upper solve's backward step with U^T instead of U
    "potrs_upper_backward_transposed": (
        "B[r * ldb + q] = pfms(B[r * ldb + q], U[r * lda + c], B[c * ldb + q]);",
        "B[r * ldb + q] = pfms(B[r * ldb + q], U[c * lda + r], B[c * ldb + q]);"),
    # a zero pivot stops the panel's updates too
    "zero_pivot_skips_update": (
        """        if (*info == 0) *info = (int32_t)(c + 1);
      } else {""",
        """        if (*info == 0) *info = (int32_t)(c + 1);
        continue;
      } else {"""),
}


def _build_mutant(text, d, name):
    src = os.path.join(d, name + ".c")
    with open(src, "w") as f:
        f.write(text)
    lib = os.path.join(d, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-I",
                           os.path.join(ROOT, "oracle"), "-o", lib,
                           os.path.join(ROOT, "oracle", "posit_oracle.c"), src, "-lm"])
    return _Lib(ctypes.CDLL(lib))


def _first_caught(lib):
    for case in CASES:
        bad = _lu_mismatch(lib, case)
        if bad:
            return case, bad
    for case in CHOL_CASES:
        bad = _chol_mismatch(lib, case)
        if bad:
            return case, bad
    return None


def test_unmutated_ref_lapack_passes():
    with tempfile.TemporaryDirectory() as d:
        assert _first_caught(_build_mutant(open(REF).read(), d, "orig")) is None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_ref_lapack_mutant_is_caught(name):
    old, new = MUTANTS[name]
    text = open(REF).read()
    assert text.count(old) == 1, f"mutation site not found for {name}"
    with tempfile.TemporaryDirectory() as d:
        assert _first_caught(_build_mutant(text.replace(old, new), d, name)) is not None, \
            f"mutant {name} survived the schedule pin"
