"""GPU parity of the variable-size batched factorisations and solves: every
system of a batch must equal the oracle's single-matrix result bit for bit
(factors, pivots, info and solutions), whatever its neighbours in the batch."""
import numpy as np
import pytest

import oracle as O
from tests.helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2401_14117_amd import posit32
    posit32.lib()
    return posit32


def p32(x):
    return O.vec_from_double(np.asarray(x, dtype=np.float64))


def _diff(a, b):
    bad = np.argwhere(a != b)
    return [(tuple(i), hex(a[tuple(i)]), hex(b[tuple(i)])) for i in bad[:6]]


def _lu_matrix(rng, n):
    return p32(rng.uniform(-1, 1, (n, n)) * 2.0 ** rng.integers(-3, 4, (n, n)))


def _spd_matrix(rng, n):
    Bm = rng.uniform(-1, 1, (n, n))
    return p32(Bm @ Bm.T / max(n, 1) + np.eye(n))


def _run_gesv(P, mats, rhss, nb, fused=True):
    import torch
    As = [to_dev(a) for a in mats]
    Bs = [to_dev(b) for b in rhss]
    vb = P.VBatch(As, Bs, lu=True)
    if fused:
        vb.gesv(nb)
    else:
        vb.getrf(nb)
        torch.cuda.synchronize()
        info_f = vb.info.clone()
        vb.getrs()
        vb.info.copy_(torch.where(info_f != 0, info_f, vb.info))
    torch.cuda.synchronize()
    return ([from_dev(a) for a in As], [p.cpu().numpy()[:a.shape[0]] for p, a in zip(vb.ipivs, mats)],
            vb.info.cpu().numpy(), [from_dev(b) for b in Bs])


def _run_posv(P, mats, rhss, nb, fused=True):
    import torch
    As = [to_dev(a) for a in mats]
    Bs = [to_dev(b) for b in rhss]
    vb = P.VBatch(As, Bs, lu=False)
    if fused:
        vb.posv(nb)
    else:
        vb.potrf(nb)
        torch.cuda.synchronize()
        info_f = vb.info.clone()
        vb.potrs()
        vb.info.copy_(torch.where(info_f != 0, info_f, vb.info))
    torch.cuda.synchronize()
    return [from_dev(a) for a in As], vb.info.cpu().numpy(), [from_dev(b) for b in Bs]


SIZES = [1, 2, 5, 16, 31, 32, 33, 64, 100, 255, 256, 257, 300, 512]


@pytest.mark.parametrize("fused", [True, False])
def test_lu_vbatched_parity(P, fused):
    rng = np.random.default_rng(11)
    sizes = sorted(SIZES, reverse=True)
    mats = [_lu_matrix(rng, n) for n in sizes]
    rhss = [p32(rng.uniform(-1, 1, (n, int(rng.integers(1, 17))))) for n in sizes]
    gA, gpiv, ginfo, gB = _run_gesv(P, mats, rhss, 256, fused)
    for i, n in enumerate(sizes):
        LU, ipiv, info = O.getrf(mats[i], 256)
        assert ginfo[i] == info == 0, (n, ginfo[i], info)
        assert np.array_equal(gpiv[i], ipiv), n
        assert np.array_equal(gA[i], LU), (n, _diff(gA[i], LU))
        X = O.getrs(LU, ipiv, rhss[i])
        assert np.array_equal(gB[i], X), (n, _diff(gB[i], X))


@pytest.mark.parametrize("fused", [True, False])
def test_chol_vbatched_parity(P, fused):
    rng = np.random.default_rng(12)
    sizes = sorted(SIZES, reverse=True)
    mats = [_spd_matrix(rng, n) for n in sizes]
    rhss = [p32(rng.uniform(-1, 1, (n, int(rng.integers(1, 17))))) for n in sizes]
    gA, ginfo, gB = _run_posv(P, mats, rhss, 256, fused)
    for i, n in enumerate(sizes):
        L, info = O.potrf(mats[i], 256)
        assert ginfo[i] == info == 0, (n, ginfo[i], info)
        # only the lower triangle is defined; the strict upper one is untouched
        assert np.array_equal(np.tril(gA[i]), np.tril(L)), (n, _diff(np.tril(gA[i]), np.tril(L)))
        assert np.array_equal(np.triu(gA[i], 1), np.triu(mats[i], 1)), n
        X = O.potrs(L, rhss[i])
        assert np.array_equal(gB[i], X), (n, _diff(gB[i], X))


def test_vbatched_other_block_size(P):
    """nb = 64: the panel and block boundaries move; still the oracle's bits."""
    rng = np.random.default_rng(13)
    sizes = [200, 130, 64, 65, 7]
    mats = [_lu_matrix(rng, n) for n in sizes]
    rhss = [p32(rng.uniform(-1, 1, (n, 2))) for n in sizes]
    gA, gpiv, ginfo, gB = _run_gesv(P, mats, rhss, 64)
    for i in range(len(sizes)):
        LU, ipiv, info = O.getrf(mats[i], 64)
        assert np.array_equal(gA[i], LU) and np.array_equal(gpiv[i], ipiv) and ginfo[i] == info
        assert np.array_equal(gB[i], O.getrs(LU, ipiv, rhss[i]))
    spd = [_spd_matrix(rng, n) for n in sizes]
    gA, ginfo, gB = _run_posv(P, spd, rhss, 64)
    for i in range(len(sizes)):
        L, info = O.potrf(spd[i], 64)
        assert np.array_equal(np.tril(gA[i]), np.tril(L)) and ginfo[i] == info == 0
        assert np.array_equal(gB[i], O.potrs(L, rhss[i]))


def test_lu_vbatched_singular_and_nar(P):
    rng = np.random.default_rng(14)
    sing = _lu_matrix(rng, 40)
    sing[:, 7] = 0                                  # zero column: info = 8
    nar = _lu_matrix(rng, 40)
    nar[3, 5] = 0x80000000
    late = _lu_matrix(rng, 300)
    late[:, 290] = 0                                # zero pivot in the second panel
    mats = [late, sing, nar]
    rhss = [p32(rng.uniform(-1, 1, (m.shape[0], 3))) for m in mats]
    gA, gpiv, ginfo, gB = _run_gesv(P, mats, rhss, 256)
    for i, m in enumerate(mats):
        LU, ipiv, info = O.getrf(m, 256)
        assert ginfo[i] == info, (i, ginfo[i], info)
        assert np.array_equal(gA[i], LU) and np.array_equal(gpiv[i], ipiv), i
        if info > 0:                                # not solved
            assert np.array_equal(gB[i], rhss[i]), i
        else:
            assert np.array_equal(gB[i], O.getrs(LU, ipiv, rhss[i])), i
    assert ginfo[0] == 291 and ginfo[1] == 8 and ginfo[2] == 0


@pytest.mark.parametrize("bad", [0, 5, 31, 32, 40, 255, 256, 300, 399])
def test_chol_vbatched_not_positive_definite(P, bad):
    """A failed diagonal leaves exactly the unblocked order's partial state,
    wherever it falls relative to the sub-blocks and blocks."""
    rng = np.random.default_rng(15)
    n = 400
    A = np.asarray(rng.uniform(-1, 1, (n, n)))
    A = A @ A.T / n + np.eye(n)
    A[bad, bad] = -50.0
    Ap = p32(A)
    good = _spd_matrix(rng, 50)
    mats = [Ap, good]
    rhss = [p32(np.ones((n, 1))), p32(np.ones((50, 1)))]
    gA, ginfo, gB = _run_posv(P, mats, rhss, 256)
    L, info = O.potrf(Ap, 256)
    assert info > 0 and ginfo[0] == info
    assert np.array_equal(gA[0], L), _diff(gA[0], L)
    assert np.array_equal(gB[0], rhss[0])           # not solved
    L2, info2 = O.potrf(good, 256)
    assert ginfo[1] == info2 == 0 and np.array_equal(np.tril(gA[1]), np.tril(L2))


def _factor_like(rng, n, diag_scale=0.0, off_lo=-27, off_hi=-7):
    """Well-conditioned stand-in factors (the solves take any matrix as L and
    U): diagonal |d| in [1, 2) 2^diag_scale, off-diagonal entries with scales
    spread over 2^off_lo .. 2^off_hi, so that the substitutions neither
    overflow nor cancel and a special value stays where it is put."""
    M = rng.uniform(0.5, 1.0, (n, n)) * rng.choice([-1.0, 1.0], (n, n)) * 2.0 ** rng.integers(off_lo, off_hi + 1, (n, n))
    np.fill_diagonal(M, rng.uniform(1.0, 2.0, n) * rng.choice([-1.0, 1.0], n) * 2.0 ** diag_scale)
    return p32(M)


@pytest.mark.parametrize("kind", ["lu", "chol"])
def test_vbatched_solve_special_values(P, kind):
    """The batched substitutions alone (the factors given) against the oracle,
    and the single-matrix substitutions on the same inputs, across 64-row
    block boundaries: a NaR right-hand side, an all-zero right-hand side
    (zero quotients, taken by the exact division), a zero and a NaR
    coefficient on row 0 (LU: only x_0 becomes NaR), a NaR diagonal
    (Cholesky: every entry NaR), quotients of 2^100 .. 2^110, beyond the
    fast range, right-hand sides with scales over 2^-30 .. 2^30."""
    import torch
    rng = np.random.default_rng(20 if kind == "lu" else 21)
    sizes = [130, 65, 64, 5, 70, 66]
    nrhs = [3, 3, 9, 1, 3, 9]
    mats, rhss, pivs = [], [], []
    for i, (n, r) in enumerate(zip(sizes, nrhs)):
        # system 2: diagonals near 2^-100 (LU's U) or 2^-50 (L, divided by twice), so
        # that the quotients reach 2^100 .. 2^110, beyond the fast range
        tiny = -100.0 if kind == "lu" else -50.0
        F = _factor_like(rng, n, diag_scale=tiny if i == 2 else 0.0, off_lo=-130 if i == 2 else -27,
                         off_hi=-120 if i == 2 else -7)
        B = p32(rng.uniform(-1, 1, (n, r)) * 2.0 ** (10 if i == 2 else rng.integers(-30, 31, (n, r))))
        if i == 0:
            B[100, 1] = 0x80000000                      # NaR right-hand side (column 1 only)
            B[:, 2] = 0                                 # zero right-hand side
        if i == 1:
            if kind == "lu":
                F[0, 0] = 0                             # zero diagonal: x_0 = NaR
                F[0, 64] = 0x80000000                   # NaR coefficient in row 0
            else:
                F[64, 64] = 0x80000000                  # NaR diagonal
        if i == 4:
            B[rng.integers(0, n, 12), rng.integers(0, r, 12)] = 0
        mats.append(F)
        rhss.append(B)
        pivs.append(np.array([int(rng.integers(c, n)) for c in range(n)], dtype=np.int32))
    As = [to_dev(a) for a in mats]
    Bs = [to_dev(b) for b in rhss]
    vb = P.VBatch(As, Bs, lu=kind == "lu")
    if kind == "lu":
        for dst, pv in zip(vb.ipivs, pivs):
            dst.copy_(torch.from_numpy(pv))
        vb.getrs()
    else:
        vb.potrs()
    torch.cuda.synchronize()
    assert list(vb.info.cpu().numpy()) == [0] * len(sizes)
    for i in range(len(sizes)):
        want = O.getrs(mats[i], pivs[i], rhss[i]) if kind == "lu" else O.potrs(mats[i], rhss[i])
        got = from_dev(Bs[i])
        assert np.array_equal(got, want), (i, _diff(got, want))
        # the single-matrix substitutions on the same inputs
        Bd = to_dev(rhss[i])
        if kind == "lu":
            P.getrs(to_dev(mats[i]), torch.from_numpy(pivs[i]).cuda(), Bd)
        else:
            P.potrs(to_dev(mats[i]), Bd)
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(Bd), want), (i, _diff(from_dev(Bd), want))


def test_vbatched_invalid_systems(P):
    """Invalid systems get a negative info and are left untouched; the rest of
    the batch is unaffected."""
    import torch
    rng = np.random.default_rng(16)
    mats = [_lu_matrix(rng, n) for n in (20, 10, 30)]
    rhss = [p32(rng.uniform(-1, 1, (m.shape[0], 2))) for m in mats]
    As = [to_dev(a) for a in mats]
    Bs = [to_dev(b) for b in rhss]
    vb = P.VBatch(As, Bs, lu=True)
    vb.max_n = 25                                   # system 2 (n = 30) exceeds it
    vb.lda[1] = 5                                   # system 1: lda < n
    vb.gesv(256)
    torch.cuda.synchronize()
    info = vb.info.cpu().numpy()
    assert list(info) == [0, -3, -1]
    assert np.array_equal(from_dev(As[1]), mats[1]) and np.array_equal(from_dev(Bs[1]), rhss[1])
    assert np.array_equal(from_dev(As[2]), mats[2]) and np.array_equal(from_dev(Bs[2]), rhss[2])
    LU, ipiv, _ = O.getrf(mats[0], 256)
    assert np.array_equal(from_dev(As[0]), LU)
    assert np.array_equal(from_dev(Bs[0]), O.getrs(LU, ipiv, rhss[0]))


def test_vbatched_empty_and_zero_sizes(P):
    import torch
    vb = P.VBatch([], None, lu=True, device=torch.device("cuda"))
    vb.getrf(256)
    mats = [np.zeros((0, 0), np.uint32), _lu_matrix(np.random.default_rng(17), 3)]
    rhss = [np.zeros((0, 1), np.uint32), p32(np.ones((3, 1)))]
    gA, gpiv, ginfo, gB = _run_gesv(P, mats, rhss, 256)
    assert list(ginfo) == [0, 0]
    LU, ipiv, _ = O.getrf(mats[1], 256)
    assert np.array_equal(gA[1], LU) and np.array_equal(gB[1], O.getrs(LU, ipiv, rhss[1]))


def test_vbatched_matches_single_matrix_calls(P):
    """Against the single-matrix GPU calls (themselves oracle-checked) on a
    larger random-size batch."""
    import torch
    rng = np.random.default_rng(18)
    sizes = sorted(np.round(np.exp(rng.uniform(np.log(16), np.log(512), 40))).astype(int),
                   reverse=True)
    mats = [_lu_matrix(rng, int(n)) for n in sizes]
    rhss = [p32(rng.uniform(-1, 1, (int(n), int(rng.integers(1, 17))))) for n in sizes]
    gA, gpiv, ginfo, gB = _run_gesv(P, mats, rhss, 256)
    for i, m in enumerate(mats):
        Ad = to_dev(m)
        _, ipiv, info = P.getrf(Ad, 256)
        Bd = to_dev(rhss[i])
        P.getrs(Ad, ipiv, Bd)
        torch.cuda.synchronize()
        assert int(info.item()) == ginfo[i]
        assert np.array_equal(from_dev(Ad), gA[i]) and np.array_equal(ipiv.cpu().numpy(), gpiv[i])
        assert np.array_equal(from_dev(Bd), gB[i])


def test_vbatched_graph_replay(P):
    """The batched solve captured in a graph: every replay (inputs restored
    eagerly between replays) equals the eager result."""
    import torch
    rng = np.random.default_rng(19)
    sizes = [150, 90, 40, 12]
    mats = [_lu_matrix(rng, n) for n in sizes]
    rhss = [p32(rng.uniform(-1, 1, (n, 4))) for n in sizes]
    eA, epiv, einfo, eB = _run_gesv(P, mats, rhss, 256)
    As = [to_dev(a) for a in mats]
    Bs = [to_dev(b) for b in rhss]
    A0 = [a.clone() for a in As]
    B0 = [b.clone() for b in Bs]
    vb = P.VBatch(As, Bs, lu=True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        vb.gesv(256)                                # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        vb.gesv(256)
    for _ in range(3):
        for a, a0 in zip(As, A0):
            a.copy_(a0)
        for b, b0 in zip(Bs, B0):
            b.copy_(b0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(sizes)):
            assert np.array_equal(from_dev(As[i]), eA[i]) and np.array_equal(from_dev(Bs[i]), eB[i])
        assert np.array_equal(vb.info.cpu().numpy(), einfo)


@pytest.mark.parametrize("kind,count", [("lu", 48), ("chol", 24)])
def test_vbatched_workload_sample(P, kind, count):
    """Systems of the batched workload itself (its size law and matrix recipe)
    with 48 <= n <= 256, where every factorisation runs blocked updates,
    batched together and each checked against the oracle bit for bit."""
    from paper_2401_14117_amd import workloads as W
    n, nrhs = W.batch_sizes(20000)
    pick = np.nonzero((n >= 48) & (n <= 256))[0][:count]
    mats, rhss = [], []
    for i in pick:
        _, A, B = next(W.batch_matrices(kind, n, nrhs, start=int(i), stop=int(i) + 1))
        mats.append(p32(A))
        rhss.append(p32(B))
    order = sorted(range(count), key=lambda j: -mats[j].shape[0])
    mats = [mats[j] for j in order]
    rhss = [rhss[j] for j in order]
    if kind == "lu":
        gA, gpiv, ginfo, gB = _run_gesv(P, mats, rhss, 256)
    else:
        gA, ginfo, gB = _run_posv(P, mats, rhss, 256)
    for j, A in enumerate(mats):
        if kind == "lu":
            F, ipiv, info = O.getrf(A, 256)
            assert np.array_equal(gpiv[j], ipiv), j
            assert np.array_equal(gA[j], F), (A.shape, _diff(gA[j], F))
            X = O.getrs(F, ipiv, rhss[j])
        else:
            F, info = O.potrf(A, 256)
            assert np.array_equal(np.tril(gA[j]), np.tril(F)), (A.shape, _diff(np.tril(gA[j]), np.tril(F)))
            X = O.potrs(F, rhss[j])
        assert ginfo[j] == info == 0, (A.shape, ginfo[j], info)
        assert np.array_equal(gB[j], X), (A.shape, _diff(gB[j], X))


def test_vbatched_large_batch_sample(P):
    """A batch of 4,000 systems, many more than the device holds resident at
    once, so most workgroups start only after others have retired; systems
    sampled across the whole batch (the last ones included) equal the
    oracle bit for bit."""
    rng = np.random.default_rng(21)
    count = 4000
    sizes = sorted(np.round(np.exp(rng.uniform(np.log(16), np.log(96), count))).astype(int),
                   reverse=True)
    mats = [_lu_matrix(rng, int(n)) for n in sizes]
    rhss = [p32(rng.uniform(-1, 1, (int(n), int(rng.integers(1, 5))))) for n in sizes]
    gA, gpiv, ginfo, gB = _run_gesv(P, mats, rhss, 256)
    assert ginfo.shape == (count,)
    picks = sorted(set(np.linspace(0, count - 1, 30).astype(int).tolist()) | {count - 2, count - 1})
    for i in picks:
        LU, ipiv, info = O.getrf(mats[i], 256)
        assert ginfo[i] == info, (i, ginfo[i], info)
        assert np.array_equal(gpiv[i], ipiv), i
        assert np.array_equal(gA[i], LU), (i, sizes[i], _diff(gA[i], LU))
        X = O.getrs(LU, ipiv, rhss[i])
        assert np.array_equal(gB[i], X), (i, sizes[i], _diff(gB[i], X))
