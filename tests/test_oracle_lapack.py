"""Pins for the oracle's blocked factorisations and solves."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from paper_2401_14117_amd import workloads as W

NAR = 0x80000000


def p32(x):
    return O.vec_from_double(np.asarray(x, dtype=np.float64))


def d64(p):
    return O.vec_to_double(p)


def _perm_from_ipiv(ipiv):
    perm = np.arange(len(ipiv))
    for c, p in enumerate(ipiv):
        perm[[c, p]] = perm[[p, c]]
    return perm


def _exact_lu(n, rng):
    """Unit lower L with entries in {0, +-1/2, +-1/4} and upper U with small
    integer entries and diagonal in {+-1, +-2, +-4}: every intermediate of the
    factorisation of A = L U is a short dyadic number, exact in Posit(32,2),
    and |L| < 1 makes partial pivoting keep the diagonal."""
    L = np.tril(rng.choice([0.0, 0.5, -0.5, 0.25, -0.25], (n, n)), -1) + np.eye(n)
    U = np.triu(rng.integers(-3, 4, (n, n)).astype(float), 1)
    U += np.diag(rng.choice([1.0, -1.0, 2.0, -2.0, 4.0, -4.0], n))
    return L, U


@pytest.mark.parametrize("n,nb", [(8, 4), (37, 16), (70, 32), (130, 64)])
def test_getrf_exact_recovery(n, nb):
    rng = np.random.default_rng(n)
    L, U = _exact_lu(n, rng)
    A = L @ U
    assert np.max(np.abs(A)) < 2 ** 20
    LU, ipiv, info = O.getrf(p32(A), nb)
    assert info == 0
    assert np.array_equal(ipiv, np.arange(n))
    got = d64(LU)
    assert np.array_equal(np.tril(got, -1), np.tril(L, -1))
    assert np.array_equal(np.triu(got), U)
    # rows shuffled: pivoting finds the permutation and the same factors
    perm = rng.permutation(n)
    LU2, ipiv2, info2 = O.getrf(p32(A[perm]), nb)
    assert info2 == 0
    assert np.array_equal(LU2, LU)
    assert np.array_equal(perm[_perm_from_ipiv(ipiv2)], np.arange(n))
    # exact solve: integer x, b = A x
    x = rng.integers(-5, 6, (n, 2)).astype(float)
    X = O.getrs(LU2, ipiv2, p32(A[perm] @ x))
    assert np.array_equal(d64(X), x)


@pytest.mark.parametrize("n,nb", [(8, 4), (37, 16), (70, 32)])
def test_getrs_trans_exact_recovery(n, nb):
    """A^T x = b with P A = L U from exact factors and shuffled rows: every
    intermediate (U^-T b = L^T P x, then P x) is a short dyadic number, so the
    integer x comes back exactly, with the interchanges undone in reverse."""
    rng = np.random.default_rng(300 + n)
    L, U = _exact_lu(n, rng)
    perm = rng.permutation(n)
    A = (L @ U)[perm]
    LU, ipiv, info = O.getrf(p32(A), nb)
    assert info == 0
    assert not np.array_equal(ipiv, np.arange(n))
    x = rng.integers(-5, 6, (n, 3)).astype(float)
    X = O.getrs(LU, ipiv, p32(A.T @ x), trans=True)
    assert np.array_equal(d64(X), x)
    # the untransposed solve of the same factors is a different system
    X2 = O.getrs(LU, ipiv, p32(A @ x))
    assert np.array_equal(d64(X2), x)


@pytest.mark.parametrize("n,nb", [(9, 4), (40, 16), (100, 32)])
def test_potrf_upper_exact_recovery(n, nb):
    """A = U^T U with U upper, positive integer diagonal in {1, 2, 4}: the
    factor comes back exactly in the upper triangle; the strict lower triangle
    (filled with NaR, which would poison any use) is neither read nor written."""
    rng = np.random.default_rng(200 + n)
    U = np.triu(rng.integers(-2, 3, (n, n)).astype(float), 1) + np.diag(rng.choice([1.0, 2.0, 4.0], n))
    A = U.T @ U
    Ap = p32(A)
    Ap[np.tril_indices(n, -1)] = NAR
    Uf, info = O.potrf(Ap, nb, upper=True)
    assert info == 0
    assert np.array_equal(np.triu(d64(Uf)), U)
    assert np.all(Uf[np.tril_indices(n, -1)] == NAR)
    x = rng.integers(-5, 6, (n, 2)).astype(float)
    X = O.potrs(Uf, p32(A @ x), upper=True)
    assert np.array_equal(d64(X), x)


def test_potrf_upper_residual_and_info():
    case = W.chol_case(150)
    A = p32(case.A)
    Uf, info = O.potrf(A, 64, upper=True)
    assert info == 0
    U = np.triu(d64(Uf))
    Ad = d64(A)
    res = np.linalg.norm(np.triu(Ad - U.T @ U)) / np.linalg.norm(Ad)
    assert res < 200 * 2.0 ** -27
    S = np.eye(10) * 2.0
    S[6, 6] = -1.0
    Sf, info = O.potrf(p32(S), 4, upper=True)
    assert info == 7
    assert np.array_equal(d64(Sf)[7:, 7:], S[7:, 7:])   # untouched after the stop


@pytest.mark.parametrize("n,nb", [(9, 4), (40, 16), (100, 32)])
def test_potrf_exact_recovery(n, nb):
    """A = L L^T with L lower, positive integer diagonal in {1, 2, 4} and small
    integer entries: square roots and quotients are exact."""
    rng = np.random.default_rng(100 + n)
    L = np.tril(rng.integers(-2, 3, (n, n)).astype(float), -1) + np.diag(rng.choice([1.0, 2.0, 4.0], n))
    A = L @ L.T
    assert np.max(np.abs(A)) < 2 ** 20
    Lf, info = O.potrf(p32(A), nb)
    assert info == 0
    assert np.array_equal(np.tril(d64(Lf)), L)
    # the strict upper triangle is untouched
    assert np.array_equal(np.triu(Lf, 1), np.triu(p32(A), 1))
    x = rng.integers(-5, 6, (n, 3)).astype(float)
    X = O.potrs(Lf, p32(A @ x))
    assert np.array_equal(d64(X), x)


def test_getrf_residual_and_accuracy():
    """PA = LU to O(n eps) and a solution more accurate than binary32 LU
    (the paper's Section 5.1 finds posit LU ~0.8 digits better at sigma=1)."""
    case = W.lu_case(200)
    A = p32(case.A)
    LU, ipiv, info = O.getrf(A, 64)
    assert info == 0
    Ad = d64(A)
    L = np.tril(d64(LU), -1) + np.eye(200)
    U = np.triu(d64(LU))
    res = np.linalg.norm(Ad[_perm_from_ipiv(ipiv)] - L @ U) / np.linalg.norm(Ad)
    assert res < 200 * 2.0 ** -27
    x64 = np.linalg.solve(case.A, case.b)
    x = d64(O.getrs(LU, ipiv, p32(case.b)))
    x32 = sl.lu_solve(sl.lu_factor(case.A.astype(np.float32)), case.b.astype(np.float32))
    assert x32.dtype == np.float32                       # LAPACK sgetrf/sgetrs
    e_posit = np.linalg.norm(x - x64) / np.linalg.norm(x64)
    e_f32 = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    assert e_posit < e_f32


def test_potrf_residual_and_accuracy():
    case = W.chol_case(200)
    A = p32(case.A)
    Lf, info = O.potrf(A, 64)
    assert info == 0
    L = np.tril(d64(Lf))
    Ad = d64(A)
    res = np.linalg.norm(np.tril(Ad - L @ L.T)) / np.linalg.norm(Ad)
    assert res < 200 * 2.0 ** -27
    x64 = np.linalg.solve(case.A, case.b)
    x = d64(O.potrs(Lf, p32(case.b)))
    x32 = sl.cho_solve(sl.cho_factor(case.A.astype(np.float32), lower=True), case.b.astype(np.float32))
    assert x32.dtype == np.float32                       # LAPACK spotrf/spotrs
    assert np.linalg.norm(x - x64) < np.linalg.norm(x32 - x64)


def test_info_codes():
    rng = np.random.default_rng(7)
    A = rng.uniform(-1, 1, (12, 12))
    A[:, 5] = 0.0                          # singular: zero column
    LU, ipiv, info = O.getrf(p32(A), 4)
    assert info == 6
    S = np.eye(10) * 2.0
    S[7, 7] = -1.0                         # not positive definite at column 7
    Lf, info = O.potrf(p32(S), 4)
    assert info == 8
    assert np.array_equal(d64(Lf)[8:, 8:], S[8:, 8:])   # untouched after the stop
    S2 = p32(np.eye(6))
    S2[3, 3] = NAR
    assert O.potrf(S2, 4)[1] == 4


def test_pivot_ties_go_to_smallest_row():
    A = np.array([[1.0, 2.0, 0.0], [-3.0, 1.0, 1.0], [3.0, 0.0, 2.0]])
    LU, ipiv, info = O.getrf(p32(A), 2)
    assert ipiv[0] == 1                   # |-3| = |3|: the first of them
