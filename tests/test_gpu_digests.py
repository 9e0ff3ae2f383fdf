"""Full-size parity by digest: the GPU library's results on workloads too
large for an inline oracle run (Rgemm squares n = 1024 and 2048, factor +
solve at n = 1024 and 4096 -- both solve directions for LU --, 10^8
elementwise pairs per operation, the square root of every non-negative
pattern) hashed and compared with the SHA-256 digests of the oracle's results
that tests/golden/make_digests.py wrote on the CPU from the same seeded
inputs.  Every output element takes part: one differing bit anywhere fails."""
import hashlib
import importlib.util
import json
import os

import numpy as np
import pytest

from tests.helpers import from_dev, to_dev

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = json.load(open(os.path.join(HERE, "golden", "digests.json")))


def _maker():
    spec = importlib.util.spec_from_file_location("make_digests", os.path.join(HERE, "golden", "make_digests.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MK = _maker()


@pytest.fixture(scope="module")
def P():
    from paper_2401_14117_amd import posit32
    posit32.lib()
    return posit32


def _need(name):
    if name not in DIGESTS:
        pytest.fail(f"tests/golden/digests.json has no entry {name}; run tests/golden/make_digests.py {name}")
    return DIGESTS[name]


@pytest.mark.parametrize("n", [1024, 2048])
def test_gemm_square_digest(P, n):
    import torch
    want = _need(f"gemm_square_n{n}")
    A, B, C, al, be = MK.gemm_inputs(MK.W.gemm_square(n))
    assert MK.sha(A, B, C) == want["inputs"]
    Cd = to_dev(C)
    P.gemm(to_dev(A), to_dev(B), Cd, al, be)
    torch.cuda.synchronize()
    assert MK.sha(from_dev(Cd)) == want["C"]


@pytest.mark.parametrize("n", [1024, 4096])
def test_lu_digest(P, n):
    import torch
    want = _need(f"lu_n{n}")
    A, b = MK.lu_inputs(n)
    assert MK.sha(A, b) == want["inputs"]
    Ad = to_dev(A)
    _, ipiv, info = P.getrf(Ad, 256)
    X, XT = to_dev(b), to_dev(b)
    P.getrs(Ad, ipiv, X)
    P.getrs(Ad, ipiv, XT, trans=True)
    torch.cuda.synchronize()
    assert int(info.item()) == want["info"]
    assert MK.sha(ipiv.cpu().numpy().astype(np.int32)) == want["ipiv"]
    assert MK.sha(from_dev(Ad)) == want["LU"]
    assert MK.sha(from_dev(X)) == want["X"]
    assert MK.sha(from_dev(XT)) == want["XT"]


@pytest.mark.parametrize("n", [1024, 4096])
def test_chol_digest(P, n):
    import torch
    want = _need(f"chol_n{n}")
    A, b = MK.chol_inputs(n)
    assert MK.sha(A, b) == want["inputs"]
    Ad = to_dev(A)
    _, info = P.potrf(Ad, 256)
    X = to_dev(b)
    P.potrs(Ad, X)
    torch.cuda.synchronize()
    assert int(info.item()) == want["info"]
    assert MK.sha(np.tril(from_dev(Ad))) == want["L"]
    assert MK.sha(from_dev(X)) == want["X"]


def test_elementwise_1e8_digest(P):
    import torch
    want = _need("elementwise_1e8")
    ops = {"add": P.OP_ADD, "sub": P.OP_SUB, "mul": P.OP_MUL, "div": P.OP_DIV}
    hs = {op: hashlib.sha256() for op in ops}
    hin = hashlib.sha256()
    for c in range(MK.EW_CHUNKS):
        a, b = MK.ew_chunk(c)
        hin.update(a.tobytes())
        hin.update(b.tobytes())
        ad, bd = to_dev(a), to_dev(b)
        for op, code in ops.items():
            out = P.elementwise(code, ad, bd)
            torch.cuda.synchronize()
            hs[op].update(from_dev(out).tobytes())
    assert hin.hexdigest() == want["inputs"]
    for op in ops:
        assert hs[op].hexdigest() == want[op], op


def test_sqrt_every_nonnegative_pattern(P):
    import torch
    want = _need("sqrt_all_nonnegative")
    h = hashlib.sha256()
    for start in range(0, 1 << 31, MK.SQRT_CHUNK):
        a = torch.arange(start, start + MK.SQRT_CHUNK, dtype=torch.int64, device="cuda").to(torch.int32)
        out = P.elementwise(P.OP_SQRT, a, None)
        torch.cuda.synchronize()
        h.update(from_dev(out).tobytes())
    assert h.hexdigest() == want["sqrt"]
