"""Pins for the CPU oracle's scalar Posit(N,2) arithmetic.

The oracle is checked here against things it cannot agree with by
construction: hand-decoded encodings, the paper's stated fraction lengths, an
independent exact-rational checker that rounds by neighbour search (a
different algorithm from the oracle's bit-string rounding), exact FP64
midpoints, and algebraic invariants.
"""
import os
import random
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O
from tests import exact_checker as X

HERE = os.path.dirname(os.path.abspath(__file__))
NAR = 0x80000000


def _read_table(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip() if line.lstrip().startswith("#") else line.strip()
            if not line:
                continue
            rows.append(line.split())
    return rows


# ---- fixed encodings ---------------------------------------------------------

def test_fixed_encodings():
    rows = _read_table("p32_encodings.txt")
    assert len(rows) >= 19
    for row in rows:
        expr, pat = row[0], int(row[1], 16)
        if expr == "NaR":
            assert np.isnan(O.to_double(pat))
            assert O.from_double(float("nan")) == pat
            assert O.fields(pat)[0] == 2
            continue
        value = Fraction(eval(expr))  # noqa: S307 - fixture of literal numbers
        assert O.from_double(float(value)) == pat, expr
        assert Fraction(O.to_double(pat)) == value, expr
        # and the independent checker decodes the same pattern to the same value
        assert X.decode(32, pat) == value, expr


def test_fraction_lengths_from_paper():
    """f_s = 27 on [1,2); 0..3 bits on [1e-38,1e-30) and [1e30,1e38)."""
    rng = np.random.default_rng(5)
    for lo, hi, fmin, fmax in _read_table("fs_ranges.txt"):
        lo, hi, fmin, fmax = float(lo), float(hi), int(fmin), int(fmax)
        xs = np.exp(rng.uniform(np.log(lo), np.log(hi), 2000))
        xs = np.concatenate([xs, [lo]])
        seen = set()
        for x in xs:
            kind, s, k, e, fs, f = O.fields(O.from_double(float(x)))
            assert kind == 0 and s == 0
            assert fmin <= fs <= fmax, (x, fs)
            seen.add(fs)
        assert min(seen) == fmin and max(seen) == fmax


def test_spacing_at_one():
    """Section 4.2: the spacing of Posit(32,2) at 1 is 2^-27."""
    nxt = O.to_double(0x40000001)
    assert nxt - 1.0 == 2.0 ** -27
    assert O.add(0x40000000, O.from_double(2.0 ** -27)) == 0x40000001


def test_golden_zone_precision():
    """Section 2: inside 1e-3 < |x| < 1e3 the relative spacing of posits is
    below binary32's 2^-23 (at least 24 fraction bits)."""
    rng = np.random.default_rng(6)
    xs = np.exp(rng.uniform(np.log(1.0001e-3), np.log(0.9999e3), 5000))
    for x in xs:
        assert O.fields(O.from_double(float(x)))[4] >= 24


def test_regime_value_formula():
    """Eq. (1): k counts the regime run (k = m-1 for ones, -m for zeros),
    value = 16^k * 2^e * 1.f; f_s = 32 - m - 2 - 2 when all exponent bits fit."""
    for m in range(1, 28):
        # a run of m ones, terminator, e = 10, fraction = 1 followed by zeros
        body = "1" * m + "0" + "10" + "1"
        body = (body + "0" * 31)[:31]
        p = int("0" + body, 2)
        kind, s, k, e, fs, f = O.fields(p)
        assert (k, e, fs) == (m - 1, 2, 28 - m)
        assert O.to_double(p) == 16.0 ** (m - 1) * 4 * 1.5
        body0 = "0" * m + "1" + "10" + "1"
        body0 = (body0 + "0" * 31)[:31]
        p0 = int("0" + body0, 2)
        kind, s, k, e, fs, f = O.fields(p0)
        assert (k, e, fs) == (-m, 2, 28 - m)
        assert O.to_double(p0) == 16.0 ** (-m) * 4 * 1.5


# ---- exhaustive Posit(8,2) against the exact checker ---------------------------

def test_exhaustive_p8_all_ops():
    N = 8
    a = np.repeat(np.arange(256, dtype=np.uint32), 256)
    b = np.tile(np.arange(256, dtype=np.uint32), 256)
    got = {op: O.vec_op(op, a, b, N=N) for op in ("add", "mul", "div")}
    bad = []
    for i in range(a.size):
        ai, bi = int(a[i]), int(b[i])
        if got["add"][i] != X.add(N, ai, bi):
            bad.append(("add", ai, bi))
        if got["mul"][i] != X.mul(N, ai, bi):
            bad.append(("mul", ai, bi))
        if got["div"][i] != X.div(N, ai, bi):
            bad.append(("div", ai, bi))
    assert not bad, bad[:10]
    s = O.vec_op("sqrt", np.arange(256, dtype=np.uint32), N=N)
    for p in range(256):
        assert s[p] == X.sqrt(N, p), p


def test_p8_rounding_reading_matters():
    """The bit-string rule and 'nearest by value' disagree for Posit(8,2)
    products in the tapered region; the oracle follows the bit-string rule
    (the checker's threshold is the (N+1)-bit midpoint pattern 2U+1)."""
    N = 8
    differ = 0
    for a in range(1, 128):
        for b in range(1, 128):
            x = X.decode(N, a) * X.decode(N, b)
            P = O.mul(a, b, N=N)
            # nearest by value among the two neighbours (ties: even pattern)
            if x >= X.decode(N, 127) or x <= X.decode(N, 1):
                continue
            lo = max(p for p in range(1, 128) if X.decode(N, p) <= x)
            hi = lo + 1 if X.decode(N, lo) != x else lo
            dl, dh = x - X.decode(N, lo), X.decode(N, hi) - x
            near = lo if dl < dh or (dl == dh and lo % 2 == 0) else hi
            differ += near != P
    assert differ > 0


# ---- sampled Posit(16,2) and Posit(32,2) ---------------------------------------

def _stratified_patterns(N, count, rng):
    """Random patterns with the regime run length drawn uniformly, so that
    long regimes (tiny and huge magnitudes) are well represented."""
    out = []
    for _ in range(count):
        m = rng.randint(1, N - 1)
        lead = rng.randint(0, 1)
        body = str(lead) * m
        if m < N - 1:
            body += str(1 - lead)
        while len(body) < N - 1:
            body += str(rng.randint(0, 1))
        p = int(body, 2)
        if rng.randint(0, 1):
            p = ((1 << N) - p) & ((1 << N) - 1)
        out.append(p)
    specials = [0, 1 << (N - 1), 1, (1 << (N - 1)) - 1, (1 << N) - 1, 1 << (N - 2)]
    return out + specials


@pytest.mark.parametrize("N,count", [(16, 1500), (32, 700)])
def test_sampled_ops_vs_checker(N, count):
    rng = random.Random(1000 + N)
    pa = _stratified_patterns(N, count, rng)
    pb = _stratified_patterns(N, count, rng)
    rng.shuffle(pb)
    a = np.array(pa, dtype=np.uint32)
    b = np.array(pb, dtype=np.uint32)
    for op, ref in (("add", X.add), ("mul", X.mul), ("div", X.div)):
        got = O.vec_op(op, a, b, N=N)
        for i in range(a.size):
            assert got[i] == ref(N, int(a[i]), int(b[i])), (op, hex(a[i]), hex(b[i]))
    got = O.vec_op("sqrt", a, N=N)
    for i in range(a.size):
        assert got[i] == X.sqrt(N, int(a[i])), ("sqrt", hex(a[i]))


def test_p32_constructed_ties():
    """Exact ties in sums and products go to the even pattern."""
    one = 0x40000000
    h = O.from_double(2.0 ** -28)                 # half an ulp at 1.0
    assert O.add(one, h) == one                   # 1 + 2^-28: tie, 1.0 even
    assert O.add(0x40000001, h) == 0x40000002     # tie, rounds up to even
    a = O.from_double(1 + 2.0 ** -14)             # (1+2^-14)^2 = 1+2^-13+2^-28
    assert O.mul(a, a) == O.from_double(1 + 2.0 ** -13)
    b = O.from_double(1 + 3 * 2.0 ** -14)         # 1+3*2^-13+9*2^-28: not a tie
    assert O.mul(b, b) == X.mul(32, b, b)
    cases = [(one, h), (0x40000001, h), (a, a), (b, b)]
    # ties with f_s = 0 (m = 28): the last kept bit is an exponent bit
    for sc in range(108, 112):
        x = O.from_double(2.0 ** sc)
        y = O.from_double(2.0 ** (sc - 1))        # x + y = 1.5 * 2^sc: midpoint
        cases.append((x, y))
    for x, y in cases:
        assert O.add(x, y) == X.add(32, x, y)
        assert O.mul(x, y) == X.mul(32, x, y)


def _even_of(u):
    return np.where(u % 2 == 0, u, u + 1)


def _boundary_check(U):
    U = np.asarray(U, dtype=np.int64)
    vals = X.decode_array_f64(32, U)
    mids = X.decode_array_f64(33, 2 * U + 1)     # exact in FP64
    assert np.all(vals < mids) and np.all(mids < X.decode_array_f64(32, U + 1))
    assert np.array_equal(O.vec_from_double(vals), U.astype(np.uint32))
    assert np.array_equal(O.vec_from_double(mids), _even_of(U).astype(np.uint32))
    down = np.nextafter(mids, 0.0)
    up = np.nextafter(mids, np.inf)
    assert np.array_equal(O.vec_from_double(down), U.astype(np.uint32))
    assert np.array_equal(O.vec_from_double(up), (U + 1).astype(np.uint32))
    assert np.array_equal(O.vec_from_double(-mids), ((1 << 32) - _even_of(U)).astype(np.uint32))


def test_p32_round_boundaries_sampled():
    """For positive patterns U, the 33-bit midpoint 2U+1 rounds to the even
    of {U, U+1}, its FP64 neighbours round down/up, and values round-trip.
    Sampled: every pattern with a regime of 26+ bits, the first and last 64
    patterns of every regime length, and 300k random patterns."""
    rng = np.random.default_rng(11)
    U = [np.arange(1, 1 << 6), np.arange((1 << 31) - (1 << 6), (1 << 31) - 1)]
    for m in range(1, 31):
        start_ones = (1 << 31) - (1 << (31 - m))          # first pattern with m ones
        start_zeros = 1 << (30 - m) if m < 31 else 1       # first with m zeros
        for s in (start_ones, start_zeros):
            U.append(np.arange(max(1, s - 64), min((1 << 31) - 1, s + 64)))
    U.append(rng.integers(1, (1 << 31) - 1, 300_000))
    U = np.unique(np.concatenate(U))
    U = U[(U >= 1) & (U < (1 << 31) - 1)]
    _boundary_check(U)


@pytest.mark.slow
def test_p32_round_boundaries_exhaustive():
    for start in range(1, (1 << 31) - 1, 1 << 24):
        stop = min(start + (1 << 24), (1 << 31) - 1)
        _boundary_check(np.arange(start, stop))


@pytest.mark.slow
def test_exhaustive_p16_vs_checker_c():
    from tests.p16_exhaustive import run_exhaustive
    assert run_exhaustive() == 0


# ---- invariants (hypothesis) ----------------------------------------------------

p32 = st.integers(min_value=0, max_value=0xFFFFFFFF)


@settings(max_examples=3000, deadline=None)
@given(p32, p32)
def test_invariants(a, b):
    neg = O.neg
    nar_in = a == NAR or b == NAR
    s, m = O.add(a, b), O.mul(a, b)
    assert s == O.add(b, a)
    assert m == O.mul(b, a)
    if nar_in:
        assert s == NAR and m == NAR
        return
    assert O.add(neg(a), neg(b)) == neg(s)
    assert O.mul(neg(a), b) == neg(m)
    assert O.mul(a, 0x40000000) == a
    assert O.mul(a, 0xC0000000) == neg(a)
    assert O.add(a, neg(a)) == 0
    assert O.add(a, 0) == a
    assert O.mul(a, 0) == 0
    assert O.from_double(O.to_double(a)) == a
    # monotone rounding: posit order is signed-integer order
    sa, sb = np.int32(np.uint32(a)), np.int32(np.uint32(b))
    da, db = O.to_double(a), O.to_double(b)
    assert (da < db) == (sa < sb)
    if b != 0:
        q = O.div(a, b)
        assert O.div(neg(a), b) == neg(q)
    assert O.mul(NAR, 0) == NAR and O.div(a, 0) == NAR


@settings(max_examples=2000, deadline=None)
@given(st.floats(allow_nan=False, allow_infinity=False, width=64),
       st.floats(allow_nan=False, allow_infinity=False, width=64))
def test_from_double_monotone(x, y):
    px, py = O.from_double(x), O.from_double(y)
    ix, iy = np.int32(np.uint32(px)), np.int32(np.uint32(py))
    if x <= y:
        assert ix <= iy
    assert O.from_double(-x) == O.neg(px)
    if x != 0:
        assert px != 0 and px != NAR


def test_p16_strided_vs_checker_c():
    """Every 257th first operand against all 2^16 second operands (add, mul,
    div) plus all 2^16 square roots, against the independent C checker."""
    from tests.p16_exhaustive import run_exhaustive
    assert run_exhaustive(stride=257) == 0
