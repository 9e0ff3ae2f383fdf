"""GPU parity of the blocked factorisations and solves against the oracle,
bit for bit (factors, pivots, info and solutions)."""
import numpy as np
import pytest

import oracle as O
from paper_2401_14117_amd import workloads as W
from tests.helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu
NAR = 0x80000000


@pytest.fixture(scope="module")
def P():
    from paper_2401_14117_amd import posit32
    posit32.lib()
    return posit32


def p32(x):
    return O.vec_from_double(np.asarray(x, dtype=np.float64))


def _gpu_getrf(P, A, nb):
    import torch
    Ad = to_dev(A)
    _, ipiv, info = P.getrf(Ad, nb)
    torch.cuda.synchronize()
    return from_dev(Ad), ipiv.cpu().numpy(), int(info.cpu().item())


def _gpu_potrf(P, A, nb):
    import torch
    Ad = to_dev(A)
    _, info = P.potrf(Ad, nb)
    torch.cuda.synchronize()
    return from_dev(Ad), int(info.cpu().item())


def _diff(a, b):
    bad = np.argwhere(a != b)
    return [(tuple(i), hex(a[tuple(i)]), hex(b[tuple(i)])) for i in bad[:6]]


@pytest.mark.parametrize("n,nb", [(1, 256), (5, 256), (64, 256), (255, 256), (257, 256), (300, 64),
                                  (300, 256), (520, 256), (130, 1)])
def test_getrf_getrs_parity(P, n, nb):
    rng = np.random.default_rng(n * 31 + nb)
    A = p32(rng.uniform(-1, 1, (n, n)) * 2.0 ** rng.integers(-3, 4, (n, n)))
    LU, ipiv, info = O.getrf(A, nb)
    gLU, gipiv, ginfo = _gpu_getrf(P, A, nb)
    assert np.array_equal(gipiv, ipiv)
    assert ginfo == info
    assert np.array_equal(gLU, LU), _diff(gLU, LU)
    B = p32(rng.uniform(-1, 1, (n, 3)))
    X = O.getrs(LU, ipiv, B)
    import torch
    Bd = to_dev(B)
    P.getrs(to_dev(LU), torch.from_numpy(ipiv).cuda(), Bd)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)


def test_getrf_singular_and_nar(P):
    rng = np.random.default_rng(3)
    A = rng.uniform(-1, 1, (40, 40))
    A[:, 7] = 0.0
    A[:, 30] = 0.0
    Ap = p32(A)
    Ap[12, 20] = NAR
    LU, ipiv, info = O.getrf(Ap, 16)
    gLU, gipiv, ginfo = _gpu_getrf(P, Ap, 16)
    assert info == 8 and ginfo == 8
    assert np.array_equal(gipiv, ipiv)
    assert np.array_equal(gLU, LU), _diff(gLU, LU)


@pytest.mark.parametrize("n,nb", [(1, 256), (7, 256), (100, 256), (256, 256), (300, 64), (300, 256),
                                  (520, 256), (77, 1)])
def test_potrf_potrs_parity(P, n, nb):
    case = W.chol_case(n, nrhs=2)
    A = p32(case.A)
    L, info = O.potrf(A, nb)
    gL, ginfo = _gpu_potrf(P, A, nb)
    assert ginfo == info == 0
    assert np.array_equal(gL, L), _diff(gL, L)
    X = O.potrs(L, p32(case.b))
    Bd = to_dev(p32(case.b))
    P.potrs(to_dev(L), Bd)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)


@pytest.mark.parametrize("bad", [5, 300, 511])
def test_potrf_not_positive_definite(P, bad):
    n = 520
    case = W.chol_case(n)
    A = case.A.copy()
    A[bad, bad] = -50.0
    Ap = p32(A)
    L, info = O.potrf(Ap, 256)
    gL, ginfo = _gpu_potrf(P, Ap, 256)
    assert ginfo == info and info > 0
    assert np.array_equal(gL, L), _diff(gL, L)


def test_getrf_group_parity(P):
    """posit32_getrf_group: eight systems of different sizes (one with a zero
    column, one with a NaR) factored together, each equal to the oracle's
    factorisation bit for bit; then the same with nb = 64."""
    import torch
    sizes = [768, 1, 300, 5, 520, 64, 257, 130]
    rng = np.random.default_rng(77)
    mats = [p32(rng.uniform(-1, 1, (k, k)) * 2.0 ** rng.integers(-3, 4, (k, k))) for k in sizes]
    mats[2][:, 40] = 0                                 # info = 41
    mats[4][500, 7] = NAR
    for nb in (256, 64):
        devs = [to_dev(a) for a in mats]
        out = P.getrf_group(devs, nb)
        torch.cuda.synchronize()
        for a, (Ad, ipiv, info) in zip(mats, out):
            LU, piv, inf = O.getrf(a, nb)
            assert int(info.item()) == inf
            assert np.array_equal(ipiv.cpu().numpy(), piv)
            assert np.array_equal(from_dev(Ad), LU), _diff(from_dev(Ad), LU)


def test_getrs_group_matches_single(P):
    """posit32_getrs_group on systems of mixed sizes and right-hand-side
    counts (special factors with NaR and zero diagonals among them): every
    solution equals posit32_getrs on it alone, and the oracle's."""
    import torch
    cases = [_solve_case(n, r, w) for n, r, w in ((150, 5, "u"), (1, 1, "b"), (200, 2, "z"), (65, 70, "l"),
                                                  (64, 1, "u"), (130, 3, "b"))]
    LUs = [to_dev(M) for M, _, _ in cases]
    pivs = [torch.from_numpy(ip).cuda() for _, _, ip in cases]
    Bg = [to_dev(B) for _, B, _ in cases]
    P.getrs_group(LUs, pivs, Bg)
    for (M, B, ip), LU, pv, bg in zip(cases, LUs, pivs, Bg):
        Bs = to_dev(B)
        P.getrs(LU, pv, Bs)
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(bg), from_dev(Bs))
        assert np.array_equal(from_dev(bg), O.getrs(M, ip, B))


def test_getrf_group_matches_single_large(P):
    """A group of the serving workload's larger sizes (600..2048): every
    system bit-identical to posit32_getrf on it alone."""
    import torch
    sizes = [2048, 600, 1500, 1024, 777, 1999, 640, 1100, 900, 1300]
    rng = np.random.default_rng(78)
    mats = [P.from_f64(torch.from_numpy(rng.uniform(-1, 1, (k, k))).cuda()) for k in sizes]
    group = P.getrf_group([m.clone() for m in mats], 256)
    for m, (Ag, pg, ig) in zip(mats, group):
        As = m.clone()
        _, ps, is_ = P.getrf(As, 256)
        torch.cuda.synchronize()
        assert int(ig.item()) == int(is_.item()) == 0
        assert torch.equal(pg, ps)
        assert torch.equal(Ag, As)


def test_getrf_phases_same_bits(P):
    """The phase-timed getrf (a diagnostic) returns getrf's bits and four
    non-negative phase times."""
    import torch
    rng = np.random.default_rng(79)
    A = P.from_f64(torch.from_numpy(rng.uniform(-1, 1, (700, 700))).cuda())
    A1, A2 = A.clone(), A.clone()
    _, p1, i1 = P.getrf(A1, 256)
    _, p2, i2, ms = P.getrf_phases(A2, 256)
    torch.cuda.synchronize()
    assert torch.equal(A1, A2) and torch.equal(p1, p2) and int(i1.item()) == int(i2.item()) == 0
    assert set(ms) == {"panel", "interchanges", "u12_solve", "trailing_update"}
    assert all(v >= 0.0 for v in ms.values()) and ms["panel"] > 0.0


def test_exact_recovery_on_gpu(P):
    """Dyadic L*U with pivot-preserving |L| < 1, rows shuffled: the GPU
    returns the exact factors (closed form, independent of the oracle)."""
    n = 300
    rng = np.random.default_rng(8)
    L = np.tril(rng.choice([0.0, 0.5, -0.5, 0.25, -0.25], (n, n)), -1) + np.eye(n)
    U = np.triu(rng.integers(-3, 4, (n, n)).astype(float), 1) + np.diag(rng.choice([1.0, -2.0, 4.0], n))
    A = (L @ U)[rng.permutation(n)]
    gLU, gipiv, ginfo = _gpu_getrf(P, p32(A), 64)
    assert ginfo == 0
    got = O.vec_to_double(gLU)
    assert np.array_equal(np.tril(got, -1), np.tril(L, -1))
    assert np.array_equal(np.triu(got), U)


@pytest.mark.parametrize("kind", ["lu", "chol"])
def test_n768_parity(P, kind):
    n = 768
    if kind == "lu":
        case = W.lu_case(n)
        A = p32(case.A)
        LU, ipiv, info = O.getrf(A, 256)
        gLU, gipiv, ginfo = _gpu_getrf(P, A, 256)
        assert np.array_equal(gipiv, ipiv) and ginfo == info
        assert np.array_equal(gLU, LU), _diff(gLU, LU)
    else:
        case = W.chol_case(n)
        A = p32(case.A)
        L, info = O.potrf(A, 256)
        gL, ginfo = _gpu_potrf(P, A, 256)
        assert ginfo == info == 0
        assert np.array_equal(gL, L), _diff(gL, L)



def _solve_case(n, nrhs, where):
    """A factor and right-hand sides holding one kind of special value:
    'u': NaR in U near the top (only the rows above it turn NaR in getrs),
    'l': NaR in L, 'b': NaR in B, 'z': zero diagonal entries near the top
    and the bottom (NaR quotients)."""
    rng = np.random.default_rng(7 * n + nrhs)
    M = p32(rng.uniform(-1, 1, (n, n)) * 2.0 ** rng.integers(-4, 5, (n, n)))
    B = p32(rng.uniform(-1, 1, (n, nrhs)))
    if where == "u" and n > 3:
        M[2, max(3, n - 40)] = NAR
    elif where == "l" and n > 1:
        M[n - 1, n // 2] = NAR
    elif where == "b":
        B[n // 2, nrhs - 1] = NAR
    elif where == "z":
        M[min(5, n - 1), min(5, n - 1)] = 0
        M[n - 1, n - 1] = 0
    ipiv = np.arange(n, dtype=np.int32)
    for c in range(0, n, 7):
        ipiv[c] = rng.integers(c, n)
    return M, B, ipiv


@pytest.mark.parametrize("where", ["u", "l", "b", "z"])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (64, 1), (65, 70), (150, 5), (200, 2)])
def test_solves_with_nar_and_zero_diagonal(P, n, nrhs, where):
    """getrs and potrs on a given factor with NaR entries or zero diagonal
    entries, over one or more 64-row solve blocks with a ragged tail and
    many right-hand sides; bit for bit against the oracle."""
    import torch
    M, B, ipiv = _solve_case(n, nrhs, where)
    X = O.getrs(M, ipiv, B)
    if where == "u" and n > 64:
        assert 0 < np.count_nonzero(X == NAR) < X.size    # NaR reaches only the rows above
    Bd = to_dev(B)
    P.getrs(to_dev(M), torch.from_numpy(ipiv).cuda(), Bd)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)
    X = O.potrs(M, B)
    Bd = to_dev(B)
    P.potrs(to_dev(M), Bd)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)


@pytest.mark.parametrize("where", ["u", "l", "b", "z"])
@pytest.mark.parametrize("n,nrhs", [(1, 1), (64, 1), (65, 70), (150, 5), (200, 2)])
def test_transposed_and_upper_solves_with_nar_and_zero_diagonal(P, n, nrhs, where):
    """getrs with op = T (A^T X = B) and the upper potrs (A = U^T U) on the
    same special factors: bit for bit against the oracle."""
    import torch
    M, B, ipiv = _solve_case(n, nrhs, where)
    X = O.getrs(M, ipiv, B, trans=True)
    Bd = to_dev(B)
    P.getrs(to_dev(M), torch.from_numpy(ipiv).cuda(), Bd, trans=True)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)
    X = O.potrs(M, B, upper=True)
    Bd = to_dev(B)
    P.potrs(to_dev(M), Bd, upper=True)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)


@pytest.mark.parametrize("n,nb", [(1, 256), (5, 256), (64, 64), (257, 256), (300, 64), (520, 256)])
def test_getrs_trans_parity(P, n, nb):
    """A^T X = B with the GPU's own factors: the oracle's transposed solve
    on the same factors, bit for bit, with row interchanges everywhere."""
    import torch
    rng = np.random.default_rng(n * 17 + nb)
    A = p32(rng.uniform(-1, 1, (n, n)) * 2.0 ** rng.integers(-3, 4, (n, n)))
    gLU, gipiv, ginfo = _gpu_getrf(P, A, nb)
    LU, ipiv, info = O.getrf(A, nb)
    assert np.array_equal(gLU, LU) and np.array_equal(gipiv, ipiv) and ginfo == info
    B = p32(rng.uniform(-1, 1, (n, 4)))
    X = O.getrs(LU, ipiv, B, trans=True)
    Bd = to_dev(B)
    P.getrs(to_dev(gLU), torch.from_numpy(gipiv).cuda(), Bd, trans=True)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)


def _gpu_potrf_upper(P, A, nb):
    import torch
    Ad = to_dev(A)
    _, info = P.potrf(Ad, nb, upper=True)
    torch.cuda.synchronize()
    return from_dev(Ad), int(info.cpu().item())


def _upper_input(n, seed, bad=None):
    """The benchmark's SPD matrix with its strict lower triangle replaced by
    unrelated patterns (an upper factorisation must not read or change it)."""
    case = W.chol_case(n, nrhs=3)
    A = case.A.copy()
    if bad is not None:
        A[bad, bad] = -50.0
    Ap = p32(A)
    rng = np.random.default_rng(seed)
    il = np.tril_indices(n, -1)
    Ap[il] = rng.integers(0, 1 << 32, il[0].size, dtype=np.uint64).astype(np.uint32)
    return Ap, p32(case.b)


@pytest.mark.parametrize("n,nb", [(1, 256), (7, 256), (33, 16), (100, 256), (256, 256), (300, 64),
                                  (520, 256), (77, 1)])
def test_potrf_potrs_upper_parity(P, n, nb):
    A, B = _upper_input(n, 40 + n)
    U, info = O.potrf(A, nb, upper=True)
    gU, ginfo = _gpu_potrf_upper(P, A, nb)
    assert ginfo == info == 0
    assert np.array_equal(gU, U), _diff(gU, U)
    il = np.tril_indices(n, -1)
    assert np.array_equal(gU[il], A[il])                 # strict lower triangle unchanged
    X = O.potrs(U, B, upper=True)
    Bd = to_dev(B)
    P.potrs(to_dev(gU), Bd, upper=True)
    assert np.array_equal(from_dev(Bd), X), _diff(from_dev(Bd), X)
    # the same bits as the lower factorisation of the mirrored matrix
    Al = A.copy()
    Al[il] = A.T[il]
    gL, _ = _gpu_potrf(P, Al, nb)
    assert np.array_equal(np.triu(gU), np.triu(gL.T))


@pytest.mark.parametrize("bad", [5, 300, 511])
def test_potrf_upper_not_positive_definite(P, bad):
    A, _ = _upper_input(520, 90 + bad, bad=bad)
    U, info = O.potrf(A, 256, upper=True)
    gU, ginfo = _gpu_potrf_upper(P, A, 256)
    assert ginfo == info == bad + 1
    assert np.array_equal(gU, U), _diff(gU, U)


def _perm(ipiv):
    """Row order of P A for LAPACK-style interchanges applied in order."""
    perm = np.arange(len(ipiv))
    for c, p in enumerate(ipiv):
        perm[c], perm[p] = perm[p], perm[c]
    return perm


# Posit(32,2) unit roundoff for |x| in [2^-12, 2^12): at least 25 fraction
# bits, so a rounding's relative error is at most 2^-26.
U_POSIT = 2.0 ** -26


@pytest.mark.parametrize("n", [4096, 8192])
def test_getrf_full_size_backward_error(P, n):
    """The benchmark's LU (uniform[-1,1], nb = 256) at its full sizes, where
    the oracle is too slow: info = 0, pivots in range, and P A = L U within
    the componentwise bound of Gaussian elimination, |P A - L U| <= n u |L||U|
    (a wrong pivot or update would miss it by orders of magnitude)."""
    import torch
    case = W.lu_case(n)
    A = P.from_f64(torch.from_numpy(case.A).cuda())
    LU = A.clone()
    _, ipiv, info = P.getrf(LU, 256)
    assert int(info.item()) == 0
    piv = ipiv.cpu().numpy()
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    F = P.to_f64(LU)
    eye = torch.eye(n, dtype=torch.float64, device=F.device)
    L = torch.tril(F, -1) + eye
    U = torch.triu(F)
    PA = P.to_f64(A)[torch.from_numpy(_perm(piv)).cuda()]
    R = (PA - L @ U).abs()
    bound = n * U_POSIT * (L.abs() @ U.abs())
    ratio = float((R / bound.clamp_min(1e-300)).max())
    print(f"n = {n}: max |residual| / bound = {ratio:.3e}")
    assert ratio <= 1.0, ratio


@pytest.mark.parametrize("n", [4096, 8192])
def test_potrf_full_size_backward_error(P, n):
    """The benchmark's Cholesky (A = B B^T / n + I, nb = 256) at its full
    sizes: info = 0 and A = L L^T within |A - L L^T| <= (n + 1) u |L||L^T|
    on the lower triangle."""
    import torch
    case = W.chol_case(n)
    A = P.from_f64(torch.from_numpy(case.A).cuda())
    Lp = A.clone()
    _, info = P.potrf(Lp, 256)
    assert int(info.item()) == 0
    L = torch.tril(P.to_f64(Lp))
    R = torch.tril(P.to_f64(A) - L @ L.T.contiguous()).abs()
    bound = torch.tril((n + 1) * U_POSIT * (L.abs() @ L.abs().T.contiguous()))
    ratio = float((R / bound.clamp_min(1e-300)).max())
    print(f"n = {n}: max |residual| / bound = {ratio:.3e}")
    assert ratio <= 1.0, ratio
