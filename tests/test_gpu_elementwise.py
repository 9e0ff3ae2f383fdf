"""GPU parity of the scalar pipeline: conversions and the elementwise
Add/Mul/Div/Sqrt kernels against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle as O
from tests.helpers import from_dev, stratified_patterns, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2401_14117_amd import posit32
    posit32.lib()
    return posit32


def _pairs(seed, count):
    rng = np.random.default_rng(seed)
    a = stratified_patterns(rng, count)
    b = stratified_patterns(rng, count)
    rng.shuffle(b)
    # golden-zone magnitudes dominate real data: add uniform patterns too
    ua = rng.integers(0, 1 << 32, count, dtype=np.int64).astype(np.uint32)
    ub = rng.integers(0, 1 << 32, count, dtype=np.int64).astype(np.uint32)
    return np.concatenate([a, ua]), np.concatenate([b, ub])


@pytest.mark.parametrize("op", ["add", "sub", "mul", "div", "sqrt"])
def test_elementwise_vs_oracle(P, op):
    a, b = _pairs({"add": 1, "sub": 2, "mul": 3, "div": 4, "sqrt": 5}[op], 400_000)
    want = O.vec_op(op, a, b)
    code = {"add": P.OP_ADD, "sub": P.OP_SUB, "mul": P.OP_MUL, "div": P.OP_DIV, "sqrt": P.OP_SQRT}[op]
    got = from_dev(P.elementwise(code, to_dev(a), None if op == "sqrt" else to_dev(b)))
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(hex(a[i]), hex(b[i]), hex(got[i]), hex(want[i])) for i in bad[:8]]


def test_constructed_ties_and_boundaries(P):
    one = 0x40000000
    h = O.from_double(2.0 ** -28)
    cases = [(one, h), (0x40000001, h), (0x7FFFFFFF, 0x7FFFFFFF), (1, 1), (1, 0xFFFFFFFF),
             (0x7FFFFFFF, 0x80000001), (one, 0xC0000000)]
    for sc in range(100, 121):
        cases.append((O.from_double(2.0 ** sc), O.from_double(2.0 ** (sc - 1))))
        cases.append((O.from_double(2.0 ** -sc), O.from_double(-(2.0 ** (-sc - 1)))))
    a = np.array([c[0] for c in cases], dtype=np.uint32)
    b = np.array([c[1] for c in cases], dtype=np.uint32)
    for op, code in (("add", P.OP_ADD), ("mul", P.OP_MUL), ("div", P.OP_DIV)):
        assert np.array_equal(from_dev(P.elementwise(code, to_dev(a), to_dev(b))), O.vec_op(op, a, b)), op


def test_from_f64_vs_oracle(P):
    import torch
    rng = np.random.default_rng(9)
    x = np.concatenate([
        rng.uniform(-1, 1, 200_000),
        rng.normal(0, 1, 100_000) * 10.0 ** rng.integers(-40, 40, 100_000),
        np.ldexp(rng.uniform(1, 2, 100_000), rng.integers(-140, 140, 100_000)),
        [0.0, -0.0, np.inf, -np.inf, np.nan, 5e-324, -5e-324, 1e308, 2.0 ** 120, 2.0 ** -120],
    ])
    got = from_dev(P.from_f64(torch.from_numpy(x).cuda()))
    assert np.array_equal(got, O.vec_from_double(x))


def test_to_f64_vs_oracle(P):
    rng = np.random.default_rng(10)
    p = np.concatenate([stratified_patterns(rng, 200_000),
                        rng.integers(0, 1 << 32, 200_000, dtype=np.int64).astype(np.uint32)])
    got = P.to_f64(to_dev(p)).cpu().numpy()
    want = O.vec_to_double(p)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.array_equal(got[ok], want[ok])
