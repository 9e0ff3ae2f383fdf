"""The allocation-free LU entry point, posit32_getrf_noalloc, called through
the C ABI: factors, pivots and info equal those of posit32_getrf on the same
input, bit for bit, on two calls in a row (the second on a smaller system, so
it reuses the library's scratch after a larger call), and the smaller one
also equals the oracle."""
import numpy as np
import pytest

import oracle as O
from tests.helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu


def _factor(L, fn, A, nb):
    import torch
    from paper_2401_14117_amd import posit32
    Ad = to_dev(A)
    n = A.shape[0]
    ipiv = torch.full((n,), -7, dtype=torch.int32, device=Ad.device)
    info = torch.full((1,), -7, dtype=torch.int32, device=Ad.device)
    rc = getattr(L, fn)(posit32._stream(None), n, nb, Ad.data_ptr(), n, ipiv.data_ptr(), info.data_ptr())
    assert rc == 0, (fn, rc)
    torch.cuda.synchronize()
    return from_dev(Ad), ipiv.cpu().numpy(), int(info.item())


def test_getrf_noalloc_matches_getrf_twice():
    from paper_2401_14117_amd import posit32
    L = posit32.lib()
    rng = np.random.default_rng(4242)
    big = O.vec_from_double(rng.uniform(-1, 1, (700, 700)) * 2.0 ** rng.integers(-3, 4, (700, 700)))
    small = O.vec_from_double(rng.uniform(-1, 1, (300, 300)))
    small[:, 17] = 0                                   # a zero column: info = 18
    for A, nb in ((big, 256), (small, 64)):
        want = _factor(L, "posit32_getrf", A, nb)
        got = _factor(L, "posit32_getrf_noalloc", A, nb)
        assert got[2] == want[2]
        assert np.array_equal(got[1], want[1])
        assert np.array_equal(got[0], want[0])
    LU, ipiv, info = O.getrf(small, 64)
    assert info == 18 == got[2]
    assert np.array_equal(got[1], ipiv) and np.array_equal(got[0], LU)
