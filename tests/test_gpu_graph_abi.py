"""Graph capture of the library's calls through the C ABI on a raw HIP stream
(no torch stream or graph object in the path): the caller begins a capture
on its own stream, makes ordinary posit32_* calls, instantiates the graph and
replays it.  Every replay, with the inputs restored eagerly in between, must
equal the eager calls bit for bit."""
import ctypes

import numpy as np
import pytest

import oracle as O
from tests.helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu

ONE = 0x40000000
CAPTURE_GLOBAL = 0          # hipStreamCaptureModeGlobal


def p32(x):
    return O.vec_from_double(np.asarray(x, dtype=np.float64))


class Hip:
    """The few HIP runtime calls the test needs, from the runtime torch and
    the library already share (same shared object, loaded once)."""

    def __init__(self):
        import torch
        torch.cuda.init()
        H = ctypes.CDLL("libamdhip64.so.7")
        vp, pvp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)
        for name, args in (("hipStreamCreate", [pvp]), ("hipStreamDestroy", [vp]),
                           ("hipStreamSynchronize", [vp]), ("hipStreamBeginCapture", [vp, ctypes.c_int]),
                           ("hipStreamEndCapture", [vp, pvp]),
                           ("hipGraphInstantiate", [pvp, vp, vp, ctypes.c_char_p, ctypes.c_size_t]),
                           ("hipGraphLaunch", [vp, vp]), ("hipGraphExecDestroy", [vp]),
                           ("hipGraphDestroy", [vp])):
            f = getattr(H, name)
            f.argtypes, f.restype = args, ctypes.c_int
        self.H = H

    def ok(self, rc, what):
        assert rc == 0, f"{what} returned {rc}"


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def test_capture_replay_through_the_c_abi():
    import torch
    from paper_2401_14117_amd import posit32
    L = posit32.lib()
    hip = Hip()
    H = hip.H
    rng = np.random.default_rng(23)
    n, m, k, nrhs = 96, 80, 72, 3
    A = p32(rng.uniform(-1, 1, (m, k)))
    Bg = p32(rng.uniform(-1, 1, (k, n)))
    C = p32(rng.uniform(-1, 1, (m, n)))
    M = p32(rng.uniform(-1, 1, (n, n)) * 2.0 ** rng.integers(-3, 4, (n, n)))
    ipiv = np.arange(n, dtype=np.int32)
    for c in range(0, n, 5):
        ipiv[c] = rng.integers(c, n)
    R = p32(rng.uniform(-1, 1, (n, nrhs)))
    dA, dB, dM = to_dev(A), to_dev(Bg), to_dev(M)
    dpiv = torch.from_numpy(ipiv).cuda()
    inputs = {"C": to_dev(C), "X1": to_dev(R), "X2": to_dev(R)}
    saved = {key: t.clone() for key, t in inputs.items()}
    torch.cuda.synchronize()

    stream = ctypes.c_void_p()
    hip.ok(H.hipStreamCreate(ctypes.byref(stream)), "hipStreamCreate")

    def calls():
        d = inputs
        assert L.posit32_gemm(stream, 0, 0, m, n, k, ONE, _ptr(dA), k, _ptr(dB), n, ONE, _ptr(d["C"]), n) == 0
        assert L.posit32_getrs(stream, 1, n, nrhs, _ptr(dM), n, _ptr(dpiv), _ptr(d["X1"]), nrhs) == 0
        assert L.posit32_potrs(stream, 1, n, nrhs, _ptr(dM), n, _ptr(d["X2"]), nrhs) == 0

    def restore():
        for key, t in inputs.items():
            t.copy_(saved[key])
        torch.cuda.synchronize()

    calls()
    hip.ok(H.hipStreamSynchronize(stream), "hipStreamSynchronize")
    eager = {key: from_dev(t) for key, t in inputs.items()}
    # the eager calls are the oracle's results
    assert np.array_equal(eager["C"], O.gemm(A, Bg, C, ONE, ONE))
    assert np.array_equal(eager["X1"], O.getrs(M, ipiv, R, trans=True))
    assert np.array_equal(eager["X2"], O.potrs(M, R, upper=True))

    restore()
    graph, exe = ctypes.c_void_p(), ctypes.c_void_p()
    hip.ok(H.hipStreamBeginCapture(stream, CAPTURE_GLOBAL), "hipStreamBeginCapture")
    calls()
    hip.ok(H.hipStreamEndCapture(stream, ctypes.byref(graph)), "hipStreamEndCapture")
    hip.ok(H.hipGraphInstantiate(ctypes.byref(exe), graph, None, None, 0), "hipGraphInstantiate")
    try:
        for _ in range(3):
            restore()
            hip.ok(H.hipGraphLaunch(exe, stream), "hipGraphLaunch")
            hip.ok(H.hipStreamSynchronize(stream), "hipStreamSynchronize")
            for key, t in inputs.items():
                assert np.array_equal(from_dev(t), eager[key]), key
            # eager work of the program between replays
            _ = int(dA.sum().item())
    finally:
        H.hipGraphExecDestroy(exe)
        H.hipGraphDestroy(graph)
        H.hipStreamDestroy(stream)
