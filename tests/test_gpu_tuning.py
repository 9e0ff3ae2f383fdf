"""The batched kernels' sub-panel width (the tuning table) never changes a
result bit: every table, the built-in one, and the autotuner's choice give
the factors, pivots, info and solutions of the oracle's single-matrix
schedule."""
import numpy as np
import pytest

import oracle as O
from tests.helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu

BIG = 2**31 - 1


@pytest.fixture(scope="module")
def P():
    from paper_2401_14117_amd import posit32
    posit32.lib()
    return posit32


def p32(x):
    return O.vec_from_double(np.asarray(x, dtype=np.float64))


def _systems(kind, seed, sizes):
    rng = np.random.default_rng(seed)
    mats, rhss = [], []
    for n in sizes:
        M = rng.uniform(-1, 1, (n, n))
        mats.append(p32(M if kind == "lu" else M @ M.T / max(n, 1) + np.eye(n)))
        rhss.append(p32(rng.uniform(-1, 1, (n, int(rng.integers(1, 9))))))
    return mats, rhss


def _run(P, kind, mats, rhss, nb, tuning, tuned=True):
    import torch
    As = [to_dev(a) for a in mats]
    Bs = [to_dev(b) for b in rhss]
    vb = P.VBatch(As, Bs, lu=(kind == "lu"))
    if tuned:
        vb.run(True, True, nb, tuning=tuning)
    elif kind == "lu":
        vb.gesv(nb, tuned=False)
    else:
        vb.posv(nb, tuned=False)
    torch.cuda.synchronize()
    piv = [p.cpu().numpy()[:a.shape[0]].copy() for p, a in zip(vb.ipivs, mats)] if vb.ipivs else []
    return [from_dev(a) for a in As], piv, vb.info.cpu().numpy().copy(), [from_dev(b) for b in Bs]


SIZES = [300, 257, 200, 129, 96, 64, 63, 40, 33, 32, 17, 5, 1]


@pytest.mark.parametrize("kind", ["lu", "chol"])
def test_every_table_gives_the_same_bits(P, kind):
    mats, rhss = _systems(kind, 31 if kind == "lu" else 32, SIZES)
    ref = _run(P, kind, mats, rhss, 256, None, tuned=False)       # built-in table, dedicated call
    tables = [P.Tuning.make([BIG], [w]) for w in (1, 3, 8, 16, 33, 64)]
    tables.append(P.Tuning.make([20, 50, 100, 250, BIG], [64, 7, 16, 40, 24]))
    for t in tables:
        got = _run(P, kind, mats, rhss, 256, t)
        for r, g in zip(ref, got):
            assert all(np.array_equal(x, y) for x, y in zip(r, g)), t.to_dict()
    # and the reference is the oracle's schedule
    for i, n in enumerate(SIZES):
        if kind == "lu":
            LU, ipiv, info = O.getrf(mats[i], 256)
            assert np.array_equal(ref[0][i], LU) and np.array_equal(ref[1][i], ipiv) and ref[2][i] == info
            assert np.array_equal(ref[3][i], O.getrs(LU, ipiv, rhss[i]))
        else:
            L, info = O.potrf(mats[i], 256)
            assert np.array_equal(np.tril(ref[0][i]), np.tril(L)) and ref[2][i] == info
            assert np.array_equal(ref[3][i], O.potrs(L, rhss[i]))


def test_table_with_failing_cholesky(P):
    """A failed diagonal inside a narrow or wide sub-panel leaves the same
    partial state."""
    mats, rhss = _systems("chol", 33, [120, 90])
    mats[0][70, 70] = 0xC0000000                                  # -1 on the diagonal
    ref = _run(P, "chol", mats, rhss, 64, None, tuned=False)
    assert ref[2][0] > 0
    for w in (1, 5, 64):
        got = _run(P, "chol", mats, rhss, 64, P.Tuning.make([BIG], [w]))
        for r, g in zip(ref, got):
            assert all(np.array_equal(x, y) for x, y in zip(r, g)), w


def test_autotune_quick(P, tmp_path, monkeypatch):
    from paper_2401_14117_amd import autotune
    res = autotune.tune(kinds=("lu", "chol"), buckets=(40, BIG), ranges=((16, 40), (41, 90)),
                        counts=(24, 6), candidates=(8, 64), reps=1, log=lambda *a: None)
    assert res["identical_results"] is True
    for kind in ("lu", "chol"):
        assert res[kind]["max_n"] == [40, BIG]
        assert all(s in (8, 64) for s in res[kind]["sub"])
        assert len(res[kind]["ms"]) == 2 and all(len(r) == 2 for r in res[kind]["ms"])
    path = autotune.write(res, str(tmp_path / "t.json"))
    monkeypatch.setenv("POSIT32_TUNING", path)
    monkeypatch.setattr(P, "_tunings", None)
    t = P.active_tuning("lu")
    assert t.to_dict() == {"max_n": [40, BIG], "sub": res["lu"]["sub"]}
    monkeypatch.setattr(P, "_tunings", None)


def test_queue_uses_given_tables(P, monkeypatch):
    """A queue created with other tables returns the same solutions."""
    rng = np.random.default_rng(34)
    monkeypatch.setattr(P, "_tunings", {"lu": P.Tuning.make([BIG], [5]),
                                         "chol": P.Tuning.make([30, BIG], [64, 9])})
    q = P.Queue(device_bytes=64 << 20)
    cases = []
    for i, n in enumerate([70, 45, 12, 130]):
        kind = i % 2
        M = rng.uniform(-1, 1, (n, n))
        A = p32(M if kind == 0 else M @ M.T / n + np.eye(n))
        cases.append((kind, A, p32(rng.uniform(-1, 1, (n, 3)))))
    outs = [q.wait(q.submit(k, B, A), 60.0) for k, A, B in cases]
    q.close()
    monkeypatch.setattr(P, "_tunings", None)
    for (kind, A, B), out in zip(cases, outs):
        assert out["status"] == 0 and out["info"] == 0
        if kind == 0:
            LU, ipiv, _ = O.getrf(A, 256)
            assert np.array_equal(out["X"], O.getrs(LU, ipiv, B))
        else:
            L, _ = O.potrf(A, 256)
            assert np.array_equal(out["X"], O.potrs(L, B))
