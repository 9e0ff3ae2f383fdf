"""Pins for the oracle's Rgemm (C = alpha*op(A)*op(B) + beta*C, Eq. (2))."""
import random

import numpy as np
import pytest

import oracle as O
from tests import exact_checker as X

ONE, NAR = 0x40000000, 0x80000000


def p32(x):
    return O.vec_from_double(np.asarray(x, dtype=np.float64))


def _rand_int_matrix(rng, shape, lo=-8, hi=8):
    return rng.integers(lo, hi, size=shape, endpoint=True)


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("alpha,beta", [(1, 1), (1, 0), (0, 1), (-1, 1), (2, -1), (0, 0), (2, 2)])
def test_textbook_small_integers(ta, tb, alpha, beta):
    """Small integers with every partial result below 2^23 are exact in
    Posit(32,2), so Rgemm must equal integer matrix multiplication."""
    rng = np.random.default_rng(100 + 10 * ta + tb)
    m, n, k = 7, 5, 9
    A = _rand_int_matrix(rng, (k, m) if ta else (m, k))
    B = _rand_int_matrix(rng, (n, k) if tb else (k, n))
    C = _rand_int_matrix(rng, (m, n))
    # leading dimensions larger than the row width: embed in wider arrays
    Aw = np.zeros((A.shape[0], A.shape[1] + 3), dtype=np.uint32)
    Aw[:, :A.shape[1]] = p32(A)
    Bw = np.zeros((B.shape[0], B.shape[1] + 2), dtype=np.uint32)
    Bw[:, :B.shape[1]] = p32(B)
    opA = A.T if ta else A
    opB = B.T if tb else B
    expect = alpha * (opA @ opB) + beta * C
    got = O.gemm(Aw[:, :A.shape[1]], Bw[:, :B.shape[1]], p32(C), p32(alpha).item(),
                 p32(beta).item(), transa=bool(ta), transb=bool(tb))
    assert np.array_equal(O.vec_to_double(got), expect.astype(np.float64))


def test_accumulation_order():
    """acc starts at 0, sums ascending k, and C is added last:
    1 + (2^-28 + 2^-28) = 1 + 2^-27 exactly, whereas adding each term to C
    first would round 1 + 2^-28 to 1 twice."""
    A = p32([[2.0 ** -28, 2.0 ** -28]])
    B = p32([[1.0], [1.0]])
    C = p32([[1.0]])
    assert O.gemm(A, B, C)[0, 0] == 0x40000001
    # alternative order for contrast
    c = ONE
    for a in A[0]:
        c = O.add(c, O.mul(int(a), ONE))
    assert c == 0x40000000


def test_ascending_k_order_matters():
    """Reordering the k loop changes the bits, so the order is part of the
    definition: 2^30 + 1 - 2^30 = 0 in ascending order (1 is lost), but
    2^30 - 2^30 + 1 = 1."""
    A = p32([[2.0 ** 30, 1.0, -(2.0 ** 30)]])
    B = p32([[1.0], [1.0], [1.0]])
    zero = p32([[0.0]])
    assert O.gemm(A, B, zero)[0, 0] == 0
    A2 = p32([[2.0 ** 30, -(2.0 ** 30), 1.0]])
    assert O.gemm(A2, B, zero)[0, 0] == ONE


def _random_posits(rng, count):
    """Random Posit(32,2) patterns with regime lengths drawn uniformly."""
    out = []
    for _ in range(count):
        m = rng.randint(1, 31)
        lead = rng.randint(0, 1)
        body = str(lead) * m + (str(1 - lead) if m < 31 else "")
        while len(body) < 31:
            body += str(rng.randint(0, 1))
        p = int(body, 2)
        if rng.randint(0, 1):
            p = ((1 << 32) - p) & 0xFFFFFFFF
        out.append(p)
    return out


@pytest.mark.parametrize("seed", range(6))
def test_tiny_against_exact_checker(seed):
    """Whole Rgemm on tiny random inputs from every regime against the exact
    checker evaluating the same sequence of rounded operations."""
    rng = random.Random(seed)
    m, n, k = rng.randint(1, 5), rng.randint(1, 5), rng.randint(0, 6)
    ta, tb = rng.randint(0, 1), rng.randint(0, 1)
    # keep magnitudes moderate for half the seeds so that sums do not saturate
    if seed % 2:
        gen = lambda c: _random_posits(rng, c)  # noqa: E731
    else:
        gen = lambda c: [O.from_double(rng.uniform(-4, 4)) for _ in range(c)]  # noqa: E731
    A = np.array(gen(m * k), dtype=np.uint32).reshape((k, m) if ta else (m, k))
    B = np.array(gen(k * n), dtype=np.uint32).reshape((n, k) if tb else (k, n))
    C = np.array(gen(m * n), dtype=np.uint32).reshape(m, n)
    alpha = [ONE, O.from_double(-0.75), 0][seed % 3]
    beta = [ONE, O.from_double(1.5), 0, ONE, O.from_double(-3.0), ONE][seed]
    got = O.gemm(A, B, C, alpha, beta, transa=bool(ta), transb=bool(tb), m=m, n=n, k=k)
    opA = A.T if ta else A
    opB = B.T if tb else B
    for i in range(m):
        for j in range(n):
            ref = X.gemm_element(opA[i, :k], opB[:k, j], int(C[i, j]), alpha, beta)
            assert got[i, j] == ref, (i, j)


def test_transpose_identity_and_sign_symmetry():
    """(A B)^T = B^T A^T bitwise, and Rgemm(-A, B) = -Rgemm(A, B) (beta = 0)."""
    rng = np.random.default_rng(3)
    A = p32(rng.uniform(-1, 1, (6, 11)) * 2.0 ** rng.integers(-12, 12, (6, 11)))
    B = p32(rng.uniform(-1, 1, (11, 4)) * 2.0 ** rng.integers(-12, 12, (11, 4)))
    zeros = np.zeros((6, 4), dtype=np.uint32)
    C1 = O.gemm(A, B, zeros, beta=0)
    C2 = O.gemm(B, A, zeros.T.copy(), beta=0, transa=True, transb=True)
    assert np.array_equal(C1, C2.T)
    negA = ((np.uint64(1 << 32) - A.astype(np.uint64)) & 0xFFFFFFFF).astype(np.uint32)
    C3 = O.gemm(negA, B, zeros, beta=0)
    assert np.array_equal(C3, ((np.uint64(1 << 32) - C1.astype(np.uint64)) & 0xFFFFFFFF).astype(np.uint32))
    # permuting rows of A permutes rows of C
    perm = rng.permutation(6)
    assert np.array_equal(O.gemm(A[perm], B, zeros, beta=0), C1[perm])


def test_nar_and_special_scalars():
    rng = np.random.default_rng(4)
    A = p32(rng.uniform(-1, 1, (4, 5)))
    B = p32(rng.uniform(-1, 1, (5, 3)))
    C = p32(rng.uniform(-1, 1, (4, 3)))
    A[2, 3] = NAR
    got = O.gemm(A, B, C)
    assert np.all(got[2] == NAR) and not np.any(got[[0, 1, 3]] == NAR)
    # beta = 0: C is not read, a NaR there is ignored
    C2 = C.copy()
    C2[0, 0] = NAR
    A2 = A.copy()
    A2[2, 3] = ONE
    assert O.gemm(A2, B, C2, beta=0)[0, 0] != NAR
    # alpha = 0: A and B are not read, C = beta*C
    got = O.gemm(A, B, C, alpha=0, beta=O.from_double(2.0))
    assert np.array_equal(O.vec_to_double(got), 2 * O.vec_to_double(C))
    # k = 0 behaves like alpha = 0
    got = O.gemm(A[:, :0], B[:0, :], C, k=0)
    assert np.array_equal(got, C)


def test_entries_match_full():
    rng = np.random.default_rng(8)
    A = p32(rng.uniform(-1, 1, (20, 33)))
    B = p32(rng.uniform(-1, 1, (33, 17)))
    C = p32(rng.uniform(-1, 1, (20, 17)))
    full = O.gemm(A, B, C, alpha=O.from_double(-1.0))
    rows = rng.integers(0, 20, 50)
    cols = rng.integers(0, 17, 50)
    ent = O.gemm_entries(A, B, rows, cols, C[rows, cols], alpha=O.from_double(-1.0))
    assert np.array_equal(ent, full[rows, cols])
