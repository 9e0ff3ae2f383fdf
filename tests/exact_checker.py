"""Independent exact checker for Posit(N,2) rounding (test code).

This is deliberately a *different algorithm* from the oracle's, so that the
two can pin each other:

* decoding parses the bit string of Eq. (1) (paper, Section 2) as text and
  evaluates it with exact rationals (``fractions.Fraction``);
* rounding does not build a bit string at all.  It binary-searches the
  monotone pattern space for the adjacent posits u <= x < w (patterns U and
  U+1) and compares x with the value of the (N+1)-bit posit whose pattern is
  2U+1, which is the rounding threshold between U and U+1.  Exact ties go to
  the even pattern.  |x| >= maxpos gives maxpos, 0 < |x| <= minpos gives
  minpos, so a nonzero value never becomes 0 or NaR.

Comparisons with an exact target are made through a callback, so that
irrational targets (square roots) are compared exactly by squaring.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import numpy as np


def mask(N: int) -> int:
    return (1 << N) - 1


def nar(N: int) -> int:
    return 1 << (N - 1)


@lru_cache(maxsize=1 << 20)
def decode(N: int, p: int):
    """Exact value of an N-bit posit pattern (Fraction), or None for NaR."""
    p &= mask(N)
    if p == 0:
        return Fraction(0)
    if p == nar(N):
        return None
    negative = p >> (N - 1)
    if negative:
        p = (1 << N) - p                      # two's complement magnitude
    body = format(p, "0%db" % N)[1:]          # the N-1 bits after the sign
    lead = body[0]
    run = len(body) - len(body.lstrip(lead))  # regime run length
    k = run - 1 if lead == "1" else -run
    rest = body[run + 1:]                     # drop the terminating bit
    ebits = (rest[:2] + "00")[:2]             # missing exponent bits are 0
    fbits = rest[2:]
    e = int(ebits, 2)
    frac = Fraction(int(fbits, 2), 1 << len(fbits)) if fbits else Fraction(0)
    value = Fraction(2) ** (4 * k + e) * (1 + frac)
    return -value if negative else value


def _round_positive(N: int, cmp) -> int:
    """Pattern of the rounded positive target; cmp(v) = sign(v - target)."""
    maxpos = (1 << (N - 1)) - 1
    if cmp(decode(N, maxpos)) <= 0:
        return maxpos
    if cmp(decode(N, 1)) >= 0:
        return 1
    lo, hi = 1, maxpos             # decode(lo) < target < decode(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if cmp(decode(N, mid)) <= 0:
            lo = mid
        else:
            hi = mid
    U = lo
    if cmp(decode(N, U)) == 0:
        return U
    c = cmp(decode(N + 1, 2 * U + 1))   # threshold between U and U+1
    if c > 0:
        return U
    if c < 0:
        return U + 1
    return U if U % 2 == 0 else U + 1


def round_exact(N: int, x: Fraction) -> int:
    if x == 0:
        return 0
    ax = abs(x)
    P = _round_positive(N, lambda v: (v > ax) - (v < ax))
    return ((1 << N) - P) & mask(N) if x < 0 else P


def add(N, a, b):
    va, vb = decode(N, a), decode(N, b)
    if va is None or vb is None:
        return nar(N)
    return round_exact(N, va + vb)


def mul(N, a, b):
    va, vb = decode(N, a), decode(N, b)
    if va is None or vb is None:
        return nar(N)
    return round_exact(N, va * vb)


def div(N, a, b):
    va, vb = decode(N, a), decode(N, b)
    if va is None or vb is None or vb == 0:
        return nar(N)
    return round_exact(N, va / vb)


def sqrt(N, a):
    va = decode(N, a)
    if va is None or va < 0:
        return nar(N)
    if va == 0:
        return 0
    return _round_positive(N, lambda v: (v * v > va) - (v * v < va))


def gemm_element(a_row, b_col, c, alpha, beta):
    """One Rgemm element in the stated order, evaluated with this checker's
    own rounding: acc = 0; acc = rnd(acc + rnd(a*b)) for ascending p; then
    r = rnd(alpha*acc); result = r if beta == 0 else rnd(r + rnd(beta*c))."""
    N = 32
    if alpha == 0 or len(a_row) == 0:
        return 0 if beta == 0 else mul(N, beta, c)
    acc = 0
    for a, b in zip(a_row, b_col):
        acc = add(N, acc, mul(N, int(a), int(b)))
    r = mul(N, alpha, acc)
    return r if beta == 0 else add(N, r, mul(N, beta, c))


def decode_array_f64(N: int, pats: np.ndarray) -> np.ndarray:
    """Vectorised decode of N-bit patterns (N <= 33) to float64 (exact for
    N <= 33).  NaR maps to NaN.  Same bit-string reading as decode()."""
    p = np.asarray(pats, dtype=np.int64) & ((1 << N) - 1)
    neg = (p >> (N - 1)) & 1
    mag = np.where(neg == 1, (1 << N) - p, p) & ((1 << N) - 1)
    out = np.zeros(p.shape, dtype=np.float64)
    normal = (p != 0) & (p != (1 << (N - 1)))
    nbits = N - 1
    lead = (mag >> (nbits - 1)) & 1
    run = np.zeros(p.shape, dtype=np.int64)
    still = np.ones(p.shape, dtype=bool)
    for i in range(nbits - 1, -1, -1):        # walk the regime run
        bit = (mag >> i) & 1
        still &= bit == lead
        run += still
    k = np.where(lead == 1, run - 1, -run)
    remaining = nbits - run - 1               # bits after the terminator
    remaining = np.maximum(remaining, 0)
    e = np.zeros(p.shape, dtype=np.int64)
    for j in range(2):
        have = remaining - j > 0
        bit = np.where(have, (mag >> np.maximum(remaining - j - 1, 0)) & 1, 0)
        e = e * 2 + bit
    fs = np.maximum(remaining - 2, 0)
    f = mag & ((np.int64(1) << fs) - 1)
    val = np.ldexp((np.int64(1) << fs) + f, (4 * k + e - fs).astype(np.int32))
    out = np.where(normal, np.where(neg == 1, -val, val), out)
    out = np.where(p == (1 << (N - 1)), np.nan, out)
    return out
