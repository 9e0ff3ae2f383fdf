"""The request queue (continuous batching): every solution is bit-identical to
the same system solved alone (and to the oracle), however the requests were
batched; admission by device footprint, resident factors, failures."""
import threading

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2401_14117_amd import posit32
    posit32.lib()
    return posit32


def p32(x):
    return O.vec_from_double(np.asarray(x, dtype=np.float64))


def _lu(rng, n):
    return p32(rng.uniform(-1, 1, (n, n)))


def _spd(rng, n):
    M = rng.uniform(-1, 1, (n, n))
    return p32(M @ M.T / n + np.eye(n))


def _alone(P, kind, A, B, nb=256):
    """The same system through the single-matrix GPU calls."""
    import torch
    from tests.helpers import from_dev, to_dev
    Ad, Bd = to_dev(A), to_dev(B)
    if kind == 0:
        _, ipiv, info = P.getrf(Ad, nb)
        P.getrs(Ad, ipiv, Bd)
    else:
        _, info = P.potrf(Ad, nb)
        P.potrs(Ad, Bd)
    torch.cuda.synchronize()
    return from_dev(Bd), int(info.item())


def test_queue_mixed_requests_bitwise(P):
    """Requests of both kinds and many sizes (some above the batched-kernel
    limit), submitted from two threads at once: each solution equals the
    system solved alone."""
    rng = np.random.default_rng(21)
    sizes = [3, 40, 200, 700, 17, 512, 513, 64, 1, 90, 300, 33, 600, 128, 9, 256]
    reqs = []
    for i, n in enumerate(sizes):
        kind = i % 2
        A = _lu(rng, n) if kind == 0 else _spd(rng, n)
        B = p32(rng.uniform(-1, 1, (n, int(rng.integers(1, 9)))))
        reqs.append((kind, A, B))
    q = P.Queue(device_bytes=256 << 20, max_batch=64, nb=256, batch_max_n=512)
    tickets = [None] * len(reqs)

    def submit(idx):
        for i in idx:
            kind, A, B = reqs[i]
            tickets[i] = q.submit(kind, B, A)

    ths = [threading.Thread(target=submit, args=(range(k, len(reqs), 2),)) for k in (0, 1)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    outs = [q.wait(t, 120.0) for t in tickets]
    st = q.stats()
    q.close()
    for (kind, A, B), out in zip(reqs, outs):
        assert out is not None and out["status"] == 0 and out["info"] == 0
        X, info = _alone(P, kind, A, B)
        assert info == 0
        assert np.array_equal(out["X"], X), (kind, A.shape[0])
        assert out["submit_s"] <= out["start_s"] <= out["done_s"]
    assert st["systems_done"] == len(reqs) and st["pool_used"] == 0 and st["error"] == 0


def test_queue_mid_size_burst_bitwise(P):
    """A burst of systems with batch_max_n / 2 < n <= batch_max_n: whether a
    batch sends them through the batched kernel (four or more of them) or
    through the single-matrix routines (fewer), each solution equals the
    system solved alone."""
    rng = np.random.default_rng(23)
    sizes = [300, 480, 257, 512, 400, 333, 290]
    reqs = []
    for i, n in enumerate(sizes):
        kind = i % 2
        A = _lu(rng, n) if kind == 0 else _spd(rng, n)
        reqs.append((kind, A, p32(rng.uniform(-1, 1, (n, 2)))))
    q = P.Queue(device_bytes=256 << 20, max_batch=64, nb=256, batch_max_n=512)
    tickets = [q.submit(kind, B, A) for kind, A, B in reqs]
    outs = [q.wait(t, 120.0) for t in tickets]
    q.close()
    for (kind, A, B), out in zip(reqs, outs):
        assert out is not None and out["status"] == 0 and out["info"] == 0
        X, info = _alone(P, kind, A, B)
        assert info == 0
        assert np.array_equal(out["X"], X), (kind, A.shape[0])


def test_queue_matches_oracle(P):
    rng = np.random.default_rng(22)
    q = P.Queue(device_bytes=64 << 20)
    cases = [(0, _lu(rng, 70), p32(rng.uniform(-1, 1, (70, 3)))),
             (1, _spd(rng, 45), p32(rng.uniform(-1, 1, (45, 2))))]
    tickets = [q.submit(k, B, A) for k, A, B in cases]
    outs = [q.wait(t, 60.0) for t in tickets]
    q.close()
    LU, ipiv, _ = O.getrf(cases[0][1], 256)
    assert np.array_equal(outs[0]["X"], O.getrs(LU, ipiv, cases[0][2]))
    L, _ = O.potrf(cases[1][1], 256)
    assert np.array_equal(outs[1]["X"], O.potrs(L, cases[1][2]))


def test_queue_admission_by_footprint(P):
    """A pool that holds only a few systems at a time: everything still
    completes (admission waits for memory), in order of arrival; a system
    larger than the pool is refused at submission."""
    rng = np.random.default_rng(23)
    n = 400                                          # 0.64 MB per system
    q = P.Queue(device_bytes=2 << 20, max_batch=64)
    reqs = [(_lu(rng, n), p32(rng.uniform(-1, 1, (n, 2)))) for _ in range(8)]
    tickets = [q.submit(0, B, A) for A, B in reqs]
    outs = [q.wait(t, 120.0) for t in tickets]
    st = q.stats()
    with pytest.raises(P.Posit32Error):
        q.submit(0, p32(np.ones((1000, 1))), _lu(rng, 1000))   # 4 MB > 2 MiB pool
    q.close()
    assert st["batches"] >= 3                        # at most 3 systems fit at once
    assert st["pool_used"] == 0
    for (A, B), out in zip(reqs, outs):
        X, _ = _alone(P, 0, A, B)
        assert out["status"] == 0 and np.array_equal(out["X"], X)
    starts = [o["start_s"] for o in outs]
    assert starts == sorted(starts)


def test_queue_max_pending(P):
    """Back-pressure: with max_pending = 2 a third submission is refused with
    P32_E_BUSY and nothing is queued; once a ticket is retired by wait a
    submission is accepted again, and every accepted request is solved."""
    rng = np.random.default_rng(27)
    n = 64
    reqs = [(_lu(rng, n), p32(rng.uniform(-1, 1, (n, 2)))) for _ in range(4)]
    q = P.Queue(device_bytes=64 << 20, max_pending=2)
    t0 = q.submit(0, reqs[0][1], reqs[0][0])
    t1 = q.submit(0, reqs[1][1], reqs[1][0])
    with pytest.raises(P.Posit32Error) as e:
        q.submit(0, reqs[2][1], reqs[2][0])
    assert e.value.code == P.E_BUSY
    out0 = q.wait(t0, 60.0)
    t3 = q.submit(0, reqs[3][1], reqs[3][0])
    with pytest.raises(P.Posit32Error) as e:
        q.submit(0, reqs[2][1], reqs[2][0])      # t1 and t3 still unretired
    assert e.value.code == P.E_BUSY
    outs = [out0, q.wait(t1, 60.0), q.wait(t3, 60.0)]
    st = q.stats()
    q.close()
    assert st["pool_used"] == 0
    for (A, B), out in zip([reqs[0], reqs[1], reqs[3]], outs):
        X, _ = _alone(P, 0, A, B)
        assert out["status"] == 0 and np.array_equal(out["X"], X)


def test_queue_resident_factor(P):
    rng = np.random.default_rng(24)
    n = 150
    A = _lu(rng, n)
    B1 = p32(rng.uniform(-1, 1, (n, 2)))
    B2 = p32(rng.uniform(-1, 1, (n, 5)))
    q = P.Queue(device_bytes=64 << 20)
    first = q.wait(q.submit(0, B1, A, keep=True), 60.0)
    h = first["factor"]
    assert first["status"] == 0 and h != 0
    again = [q.submit(0, B2, factor=h) for _ in range(3)]
    outs = [q.wait(t, 60.0) for t in again]
    assert q.stats()["resident_factors"] == 1
    q.release(h)
    with pytest.raises(P.Posit32Error):
        q.submit(0, B2, factor=h)                     # released
    st = q.stats()
    q.close()
    LU, ipiv, _ = O.getrf(A, 256)
    assert np.array_equal(first["X"], O.getrs(LU, ipiv, B1))
    X2 = O.getrs(LU, ipiv, B2)
    for o in outs:
        assert o["status"] == 0 and o["factor"] == 0 and np.array_equal(o["X"], X2)
    assert st["resident_factors"] == 0 and st["pool_used"] == 0


def test_queue_large_resident_factor(P):
    """Above the batched-kernel limit the single-matrix routines serve both
    the factorisation and the later solves."""
    rng = np.random.default_rng(25)
    n = 600
    A = _spd(rng, n)
    B = p32(rng.uniform(-1, 1, (n, 3)))
    q = P.Queue(device_bytes=64 << 20, batch_max_n=512)
    first = q.wait(q.submit(1, B, A, keep=True), 60.0)
    second = q.wait(q.submit(1, B, factor=first["factor"]), 60.0)
    q.release(first["factor"])
    q.close()
    X, info = _alone(P, 1, A, B)
    assert info == 0
    assert np.array_equal(first["X"], X) and np.array_equal(second["X"], X)


def test_queue_failed_factorisation(P):
    """info > 0: the system is not solved and not kept; other requests are
    unaffected."""
    rng = np.random.default_rng(26)
    S = _lu(rng, 30)
    S[:, 4] = 0
    N = _spd(rng, 30)
    N[10, 10] = p32([-5.0])[0]
    good = _lu(rng, 30)
    B = p32(np.ones((30, 1)))
    q = P.Queue(device_bytes=64 << 20)
    ts = [q.submit(0, B, S, keep=True), q.submit(1, B, N, keep=True), q.submit(0, B, good)]
    outs = [q.wait(t, 60.0) for t in ts]
    st = q.stats()
    q.close()
    assert outs[0]["info"] == 5 and outs[0]["factor"] == 0 and np.array_equal(outs[0]["X"], B)
    assert outs[1]["info"] == O.potrf(N, 256)[1] > 0 and outs[1]["factor"] == 0
    assert outs[2]["info"] == 0 and np.array_equal(outs[2]["X"], _alone(P, 0, good, B)[0])
    assert st["resident_factors"] == 0


def test_queue_large_lu_burst_factored_together(P):
    """A burst of large LU systems (600..2048, one singular) submitted at
    once: the queue factors the new ones of a batch together (grouped
    panels and trailing updates); every solution equals the system solved
    alone, and the oracle's for two of them."""
    rng = np.random.default_rng(31)
    sizes = [2048, 600, 1500, 700, 1024, 1999, 640, 768, 1100, 900, 1300, 650, 1800, 610, 1200, 1600, 800,
             620]
    reqs = []
    for i, n in enumerate(sizes):
        A = _lu(rng, n)
        if i == 3:
            A[:, 10] = 0                                # singular: info = 11, not solved
        B = p32(rng.uniform(-1, 1, (n, int(rng.integers(1, 5)))))
        reqs.append((A, B))
    q = P.Queue(device_bytes=1 << 30, max_batch=64, nb=256, batch_max_n=512)
    tickets = [q.submit(0, B, A) for A, B in reqs]
    outs = [q.wait(t, 300.0) for t in tickets]
    st = q.stats()
    q.close()
    assert st["batches"] < len(sizes)                   # several systems shared a batch
    for i, ((A, B), out) in enumerate(zip(reqs, outs)):
        assert out is not None and out["status"] == 0
        X, info = _alone(P, 0, A, B)
        assert out["info"] == info == (11 if i == 3 else 0)
        if info == 0:
            assert np.array_equal(out["X"], X), i
        else:
            assert np.array_equal(out["X"], B)           # a failed factorisation is not solved
        if sizes[i] in (600, 768):
            LU, ipiv, _ = O.getrf(A, 256)
            assert np.array_equal(out["X"], O.getrs(LU, ipiv, B)), i


def test_queue_large_chol_burst_on_side_streams(P):
    """A burst of large Cholesky systems (520..1400, one not positive
    definite, two solved with a resident factor) submitted at once: the
    queue runs a batch's large Cholesky systems side by side on several
    streams; every solution equals the system solved alone, and the
    oracle's for one of them."""
    rng = np.random.default_rng(32)
    sizes = [1400, 520, 900, 610, 1100, 700, 530, 1250, 800, 560]
    reqs = []
    for i, n in enumerate(sizes):
        A = _spd(rng, n)
        if i == 4:
            A[300, 300] = p32([-3.0])[0]                # fails at column 301
        B = p32(rng.uniform(-1, 1, (n, int(rng.integers(1, 6)))))
        reqs.append((A, B))
    q = P.Queue(device_bytes=1 << 30, max_batch=64, nb=256, batch_max_n=512)
    first = q.wait(q.submit(1, reqs[1][1], reqs[1][0], keep=True), 120.0)
    tickets = [q.submit(1, B, A) for A, B in reqs]
    again = [q.submit(1, reqs[1][1], factor=first["factor"]) for _ in range(2)]
    outs = [q.wait(t, 300.0) for t in tickets]
    outs_again = [q.wait(t, 300.0) for t in again]
    st = q.stats()
    q.release(first["factor"])
    q.close()
    assert st["batches"] < len(sizes) + 3                # several systems shared a batch
    for i, ((A, B), out) in enumerate(zip(reqs, outs)):
        assert out is not None and out["status"] == 0
        X, info = _alone(P, 1, A, B)
        assert out["info"] == info
        assert (info > 0) == (i == 4)
        assert np.array_equal(out["X"], X if info == 0 else B), i
    X1, _ = _alone(P, 1, reqs[1][0], reqs[1][1])
    assert np.array_equal(first["X"], X1)
    for o in outs_again:
        assert o["status"] == 0 and np.array_equal(o["X"], X1)
    L, info = O.potrf(reqs[6][0], 256)
    assert info == 0 and np.array_equal(outs[6]["X"], O.potrs(L, reqs[6][1]))
