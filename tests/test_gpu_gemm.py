"""GPU parity of Rgemm (posit32_gemm) against the oracle, bit for bit."""
import functools

import numpy as np
import pytest

import oracle as O
from paper_2401_14117_amd import workloads as W
from tests.helpers import case_patterns, from_dev, stratified_patterns, to_dev

pytestmark = pytest.mark.gpu
ONE, NAR = 0x40000000, 0x80000000


@pytest.fixture(scope="module")
def P():
    from paper_2401_14117_amd import posit32
    posit32.lib()
    return posit32


def _run(P, A, B, C, alpha, beta, ta=False, tb=False):
    Cd = to_dev(C)
    P.gemm(to_dev(A), to_dev(B), Cd, alpha, beta, transa=ta, transb=tb)
    return from_dev(Cd)


def _report(got, want):
    bad = np.argwhere(got != want)
    return [(tuple(ix), hex(got[tuple(ix)]), hex(want[tuple(ix)])) for ix in bad[:6]]


def test_small_uniform_128():
    """m = n = k = 128, uniform[-1,1], seed 1, alpha = beta = 1."""
    from paper_2401_14117_amd import posit32 as P
    A, B, C, al, be = case_patterns(W.gemm_uniform(128, 128, 128, seed=1))
    want = O.gemm(A, B, C, al, be)
    got = _run(P, A, B, C, al, be)
    assert np.array_equal(got, want), _report(got, want)


@pytest.mark.parametrize("m,n,k,ta,tb", [
    (130, 67, 45, 0, 0), (67, 130, 45, 0, 1), (45, 67, 130, 1, 0), (64, 64, 64, 1, 1),
    (1, 1, 1, 0, 0), (3, 200, 17, 0, 1), (257, 129, 300, 0, 0), (129, 257, 33, 1, 1),
    (200, 3, 1, 1, 0), (65, 63, 17, 0, 0),
])
def test_ragged_scaled(P, m, n, k, ta, tb):
    """Ragged shapes spanning several tiles, magnitudes 2^-12..2^12 with a
    dense NaR/zero sprinkle, all transposes."""
    case = W.gemm_scaled(m, n, k, seed=m * 7 + n * 3 + k, sprinkle=2e-3)
    A, B, C, _, _ = case_patterns(case)
    if ta:
        A = np.ascontiguousarray(A.reshape(m, k).T)
    if tb:
        B = np.ascontiguousarray(B.reshape(k, n).T)
    al, be = O.from_double(-1.0 if k % 2 else 1.5), O.from_double(1.0 if m % 2 else -0.25)
    want = O.gemm(A, B, C, al, be, transa=bool(ta), transb=bool(tb))
    got = _run(P, A, B, C, al, be, bool(ta), bool(tb))
    assert np.array_equal(got, want), _report(got, want)


# The library picks the workgroup tile from the output shape: 64 x 32 tiles
# when there are at least four per compute unit (1024 on MI355X), else 32 x 32
# tiles when there are at least two per compute unit, else 8 x 8 tiles, with
# only checked k-steps when there are fewer than two of those per compute unit.
# The shapes below land in each regime, ragged in every dimension.
@pytest.mark.parametrize("m,n,k,ta,tb,regime", [
    (2049, 1057, 37, 0, 0, "64x32"), (1057, 2049, 19, 1, 1, "64x32"), (1100, 1901, 5, 0, 1, "64x32"),
    (700, 801, 45, 0, 0, "32x32"), (801, 700, 33, 1, 0, "32x32"), (769, 735, 17, 1, 1, "32x32"),
    (511, 513, 70, 0, 1, "8x8"), (300, 300, 70, 1, 1, "8x8"),
    (9, 2000, 65, 0, 0, "8x8 checked"), (300, 7, 100, 1, 0, "8x8 checked"), (128, 128, 128, 0, 0, "8x8 checked"),
])
def test_tile_regimes(P, m, n, k, ta, tb, regime):
    """Each workgroup-tile regime of the Rgemm launch (picked from m and n),
    all transposes, NaR/zero sprinkle, against the oracle bit for bit."""
    big = -(-m // 64) * -(-n // 32)
    mid = -(-m // 32) * -(-n // 32)
    small = -(-m // 8) * -(-n // 8)
    want_regime = ("64x32" if big >= 1024 else "32x32" if mid >= 512 else "8x8" if small >= 512
                   else "8x8 checked")
    assert want_regime == regime
    case = W.gemm_scaled(m, n, k, seed=m + 3 * n + 7 * k, sprinkle=1e-4)
    A, B, C, _, _ = case_patterns(case)
    if ta:
        A = np.ascontiguousarray(A.reshape(m, k).T)
    if tb:
        B = np.ascontiguousarray(B.reshape(k, n).T)
    al, be = O.from_double(-1.0), O.from_double(1.0 if k % 2 else 0.5)
    want = O.gemm(A, B, C, al, be, transa=bool(ta), transb=bool(tb))
    got = _run(P, A, B, C, al, be, bool(ta), bool(tb))
    assert np.array_equal(got, want), _report(got, want)


@pytest.mark.parametrize("alpha,beta", [(ONE, 0), (0, ONE), (0, 0), (NAR, ONE), (ONE, NAR),
                                        (0xC0000000, 0x48000000), (0x38000000, ONE)])
def test_alpha_beta(P, alpha, beta):
    rng = np.random.default_rng(21)
    A = O.vec_from_double(rng.uniform(-1, 1, (70, 40)))
    B = O.vec_from_double(rng.uniform(-1, 1, (40, 90)))
    C = O.vec_from_double(rng.uniform(-1, 1, (70, 90)))
    C[5, 7] = NAR
    want = O.gemm(A, B, C, alpha, beta)
    got = _run(P, A, B, C, alpha, beta)
    assert np.array_equal(got, want), _report(got, want)


def test_k_zero_and_empty(P):
    import torch
    rng = np.random.default_rng(22)
    C = O.vec_from_double(rng.uniform(-1, 1, (20, 30)))
    A = np.zeros((20, 0), dtype=np.uint32)
    B = np.zeros((0, 30), dtype=np.uint32)
    Cd = to_dev(C)
    P.gemm(torch.zeros((20, 0), dtype=torch.int32, device="cuda"),
           torch.zeros((0, 30), dtype=torch.int32, device="cuda"), Cd, ONE, 0x48000000)
    assert np.array_equal(from_dev(Cd), O.gemm(A, B, C, ONE, 0x48000000, k=0))
    # m = 0 / n = 0: nothing happens
    E = torch.zeros((0, 5), dtype=torch.int32, device="cuda")
    P.gemm(torch.zeros((0, 3), dtype=torch.int32, device="cuda"),
           torch.zeros((3, 5), dtype=torch.int32, device="cuda"), E)


def test_every_regime(P):
    """Operands from every regime length: products and sums reach the tapered
    region, saturation, f_s = 0 and minpos, exercising the exact rare path."""
    rng = np.random.default_rng(23)
    m, n, k = 40, 36, 50
    A = stratified_patterns(rng, m * k)[:m * k].reshape(m, k)
    B = stratified_patterns(rng, k * n)[:k * n].reshape(k, n)
    C = stratified_patterns(rng, m * n)[:m * n].reshape(m, n)
    want = O.gemm(A, B, C, ONE, ONE)
    got = _run(P, A, B, C, ONE, ONE)
    assert np.array_equal(got, want), _report(got, want)


def test_small_integers_exact_cancellation(P):
    """Small integers: many exact ties-free sums and exact cancellations to 0."""
    rng = np.random.default_rng(24)
    A = rng.integers(-3, 4, (96, 80))
    B = rng.integers(-3, 4, (80, 72))
    C = rng.integers(-3, 4, (96, 72))
    Ap, Bp, Cp = (O.vec_from_double(x.astype(np.float64)) for x in (A, B, C))
    got = _run(P, Ap, Bp, Cp, ONE, ONE)
    assert np.array_equal(got, O.vec_from_double((A @ B + C).astype(np.float64)))


def test_leading_dimension_padding(P):
    import torch
    rng = np.random.default_rng(25)
    Abig = O.vec_from_double(rng.uniform(-1, 1, (50, 77)))
    Bbig = O.vec_from_double(rng.uniform(-1, 1, (33, 91)))
    Cbig = O.vec_from_double(rng.uniform(-1, 1, (50, 100)))
    A, B, C = Abig[:, :33], Bbig[:, :61], Cbig[:, :61]
    want = O.gemm(A, B, C, ONE, ONE)
    Ad, Bd, Cd = to_dev(Abig), to_dev(Bbig), to_dev(Cbig)
    P.gemm(Ad[:, :33], Bd[:, :61], Cd[:, :61], ONE, ONE)
    got = from_dev(Cd)
    assert np.array_equal(got[:, :61], want)
    assert np.array_equal(got[:, 61:], Cbig[:, 61:])     # untouched


def test_deterministic(P):
    rng = np.random.default_rng(26)
    A = O.vec_from_double(rng.uniform(-1, 1, (300, 200)))
    B = O.vec_from_double(rng.uniform(-1, 1, (200, 260)))
    C = O.vec_from_double(rng.uniform(-1, 1, (300, 260)))
    r1 = _run(P, A, B, C, ONE, ONE)
    r2 = _run(P, A, B, C, ONE, ONE)
    assert np.array_equal(r1, r2)


def _sampled_rows_cols(case, rng, count):
    m, n = case.m, case.n
    rows = list(rng.integers(0, m, count)) + [0, m - 1]
    cols = list(rng.integers(0, n, count)) + [0, n - 1]
    # every row/column that holds a sprinkled special value
    for mat, axis in ((case.A, 0), (case.B, 1)):
        if mat.zero_mask is None:
            continue
        hit = np.argwhere(mat.zero_mask | mat.nar_mask)
        for ix in hit[:32]:
            if axis == 0:
                rows.append(int(ix[0])); cols.append(int(rng.integers(0, n)))
            else:
                cols.append(int(ix[1])); rows.append(int(rng.integers(0, m)))
    return np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64)


def _case(which):
    if which == "square_8192":
        return W.gemm_square(8192)
    if which.startswith("trailing_j"):
        return W.gemm_trailing(int(which[len("trailing_j"):]))
    if which.startswith("normal_sigma"):
        return W.gemm_normal(8192, float(which[len("normal_sigma"):]))
    raise ValueError(which)


@functools.lru_cache(maxsize=1)
def _square8192():
    case = W.gemm_square(8192)
    return (case,) + case_patterns(case)


@pytest.mark.parametrize("which", ["square_8192", "trailing_j1", "trailing_j8", "trailing_j16",
                                   "trailing_j24", "trailing_j30", "normal_sigma1e+06"])
def test_full_size_sampled(P, which):
    """Full-size workloads in the benchmark's launch configuration (the square
    n = 8192 case, the LU trailing-update shapes 8192 - 256 j with k = 256,
    the paper's largest-magnitude normal inputs), checked on sampled outputs
    that the oracle computes one by one."""
    import torch
    if which == "square_8192":
        case, A, B, C, al, be = _square8192()
    else:
        case = _case(which)
        A, B, C, al, be = case_patterns(case)
    Cd = to_dev(C)
    P.gemm(to_dev(A), to_dev(B), Cd, al, be)
    torch.cuda.synchronize()
    got = from_dev(Cd)
    rng = np.random.default_rng(27)
    rows, cols = _sampled_rows_cols(case, rng, 300)
    want = O.gemm_entries(A, B, rows, cols, C[rows, cols], al, be)
    bad = np.nonzero(got[rows, cols] != want)[0]
    assert bad.size == 0, [(rows[i], cols[i], hex(got[rows[i], cols[i]]), hex(want[i])) for i in bad[:6]]


def test_full_size_transposes(P):
    """NT, TN and TT at n = 8192 on the square case's matrices stored
    transposed: op(A) op(B) is the same product, so every one of the 67M
    outputs must equal the NN launch's, and sampled outputs equal the
    oracle's transposed evaluation."""
    import torch
    case, A, B, C, al, be = _square8192()
    n = case.n
    Cd = to_dev(C)
    Ad, Bd = to_dev(A), to_dev(B)
    P.gemm(Ad, Bd, Cd, al, be)
    torch.cuda.synchronize()
    nn = from_dev(Cd)
    At, Bt = np.ascontiguousarray(A.T), np.ascontiguousarray(B.T)
    Atd, Btd = to_dev(At), to_dev(Bt)
    rng = np.random.default_rng(28)
    rows, cols = _sampled_rows_cols(case, rng, 100)
    for ta, tb in ((False, True), (True, False), (True, True)):
        Cd = to_dev(C)
        P.gemm(Atd if ta else Ad, Btd if tb else Bd, Cd, al, be, transa=ta, transb=tb)
        torch.cuda.synchronize()
        got = from_dev(Cd)
        assert np.array_equal(got, nn), (ta, tb, _report(got, nn))
        want = O.gemm_entries(At if ta else A, Bt if tb else B, rows, cols, C[rows, cols], al, be,
                              transa=ta, transb=tb, k=n)
        assert np.array_equal(got[rows, cols], want), (ta, tb)
