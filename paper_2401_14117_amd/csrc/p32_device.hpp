// p32_device.hpp -- Posit(32,2) arithmetic on the gfx950 integer VALU.
//
// Format (paper, Section 2, Eq. (1)): x = (-1)^s * 16^k * 2^e * 1.f.  After
// the sign comes the regime, a run of m identical bits closed by the opposite
// bit (k = m-1 for a run of ones, k = -m for a run of zeros), then e_s = 2
// exponent bits and f_s = 28 - m fraction bits (missing exponent bits read as
// zero).  0 is the all-zero pattern, NaR is 0x80000000, negative values are
// two's complements of positive patterns.  The scale of a value is 4k + e.
//
// Results are rounded to nearest with ties to the even pattern, never to 0 or
// NaR: |x| >= maxpos = 2^120 gives maxpos and 0 < |x| <= minpos = 2^-120 gives
// minpos (the posit-standard rounding SoftPosit implements; the paper ports
// SoftPosit's add and multiply, Section 3.2).
//
// Two representations are used on the device:
//
//  * Decoded operand (from a pattern): a signed significand s with |s| in
//    [2^27, 2^28) (hidden bit at 27, fraction below it) and the scale sc, so
//    x = s * 2^(sc - 27).  Decoding happens once per element when a tile is
//    staged, not once per operation (the paper's pre-processing, Section 2).
//
//  * Window form (products and running sums): a signed 32-bit h with
//    |h| <= 2^29 and an exponent e, x = h * 2^(e - 28).  Rounded values keep
//    their significand bits at h[28..1]; e is the scale (one less for the
//    exact value -2^e' whose two's complement normalises one bit lower, which
//    never changes a result because such a value is exact).  Zero is h = 0,
//    e = EZERO.  Values stay decoded across the whole k loop; the bit pattern
//    is written once per output element (the paper's post-processing).
//
// The fast multiply and add round in this form with 64-bit two's-complement
// windows and flag the cases they do not cover (zero results, cancellation of
// more than 30 bits, scales with f_s = 0, the tapered regime |scale| >= 109,
// saturation).  Flagged lanes are recomputed by the general routines below,
// which handle every input exactly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p32 {

constexpr uint32_t kNaR = 0x80000000u;
constexpr uint32_t kOne = 0x40000000u;
constexpr uint32_t kMaxpos = 0x7FFFFFFFu;
constexpr int kEZero = -4096;     // window exponent of zero
constexpr int kMaxScale = 120;    // maxpos = 2^120, minpos = 2^-120

struct dec {
  int32_t s;    // signed significand, |s| in [2^27, 2^28); 0 for zero
  int32_t sc;   // scale 4k + e; kEZero for zero
};

struct win {
  int32_t h;    // |h| <= 2^29
  int32_t e;
};

// ---------------------------------------------------------------------------
// decoding (Section 2, Eq. (1)): count the regime run with a leading-zero
// count instead of a bit loop, so the cost does not depend on the magnitude.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool is_nar(uint32_t p) { return p == kNaR; }

__device__ __forceinline__ dec decode(uint32_t p) {
  const uint32_t neg = p >> 31;
  const uint32_t a = neg ? (0u - p) : p;          // pattern of |x|
  const uint32_t x = a << 1;                      // body, left-aligned
  const uint32_t lead = x >> 31;
  const int run = __clz(lead ? ~x : x);           // regime run length m
  const int k = lead ? run - 1 : -run;
  // bits after the terminator; a 64-bit shift gives 0 for run = 31
  const uint32_t rest = (uint32_t)((uint64_t)x << (run + 1));
  const int e = (int)(rest >> 30);
  const int32_t mag = (int32_t)((1u << 27) | ((rest << 2) >> 5));
  dec d;
  d.s = neg ? -mag : mag;
  d.sc = 4 * k + e;
  if ((p << 1) == 0u) {                           // 0 or NaR
    d.s = 0;
    d.sc = kEZero;
  }
  return d;
}

__device__ __forceinline__ win to_win(dec d) {
  win w;
  w.h = d.s * 2;
  w.e = d.s ? d.sc : kEZero;
  return w;
}

// ---------------------------------------------------------------------------
// general rounding of an exact value  (-1)^neg * (M + sticky) * 2^x  where
// sticky means "strictly above M by less than one unit".  The infinitely
// precise posit string is assembled in a 64-bit word: the N-1 = 31 bits after
// the sign land in [63:33], the guard bit in [32], everything below is sticky.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int clz128(unsigned __int128 v) {
  const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
  return hi ? __clzll(hi) : 64 + (lo ? __clzll(lo) : 64);
}

__device__ inline uint32_t round_general(bool neg, unsigned __int128 M, int x, bool sticky) {
  if (M == 0) {
    if (!sticky) return 0u;
    return neg ? 0xFFFFFFFFu : 1u;                // below one unit: minpos
  }
  const int t = 127 - clz128(M);                  // leading bit of M
  const int sc = x + t;                           // floor(log2 |value|)
  uint32_t P;
  const bool pow2 = (M & (M - 1)) == 0 && !sticky;
  if (sc >= kMaxScale) {
    P = kMaxpos;
  } else if (sc < -kMaxScale || (sc == -kMaxScale && pow2)) {
    P = 1u;
  } else {
    const int k = sc >> 2;                        // floor(sc / 4)
    const int e = sc & 3;
    const int R = k >= 0 ? k + 2 : 1 - k;         // run + terminator, <= 31
    const uint64_t regime = k >= 0 ? ((((uint64_t)1 << (k + 1)) - 1) << 1) : (uint64_t)1;
    // fraction bits of M (below its leading one), left-aligned in 128 bits
    const unsigned __int128 fr = t == 0 ? (unsigned __int128)0 : (M << (128 - t));
    const uint64_t f64 = (uint64_t)(fr >> 64);
    bool s = sticky || (uint64_t)fr != 0;
    const int fsh = R + 2;                        // <= 33
    s = s || (f64 & ((((uint64_t)1) << fsh) - 1)) != 0;
    const uint64_t body = (regime << (64 - R)) | ((uint64_t)e << (62 - R)) | (f64 >> fsh);
    P = (uint32_t)(body >> 33);
    const bool G = (body >> 32) & 1u;
    s = s || (uint32_t)body != 0;
    if (G && (s || (P & 1u))) P += 1u;
  }
  return neg ? (0u - P) : P;
}

// exact product of two decoded operands, rounded
__device__ inline uint32_t mul_general(dec a, dec b) {
  if (a.s == 0 || b.s == 0) return 0u;
  const bool neg = (a.s < 0) != (b.s < 0);
  const uint64_t ma = (uint64_t)(a.s < 0 ? -(int64_t)a.s : a.s);
  const uint64_t mb = (uint64_t)(b.s < 0 ? -(int64_t)b.s : b.s);
  return round_general(neg, (unsigned __int128)(ma * mb), a.sc + b.sc - 54, false);
}

// pattern of a window-form value that is exactly representable
__device__ inline uint32_t encode_exact(win a) {
  if (a.h == 0) return 0u;
  const bool neg = a.h < 0;
  const uint64_t m = (uint64_t)(neg ? -(int64_t)a.h : a.h);
  return round_general(neg, m, a.e - 28, false);
}

// exact sum of two window-form values (each exactly a posit), rounded
__device__ inline uint32_t add_general(win a, win b) {
  if (a.h == 0) return encode_exact(b);
  if (b.h == 0) return encode_exact(a);
  // operand 1: the one whose lowest bit has the larger weight
  win p = a, q = b;
  if (a.e < b.e) { p = b; q = a; }
  const bool n1 = p.h < 0, n2 = q.h < 0;
  const uint64_t m1 = (uint64_t)(n1 ? -(int64_t)p.h : p.h);
  const uint64_t m2 = (uint64_t)(n2 ? -(int64_t)q.h : q.h);
  const int d = p.e - q.e;                        // >= 0
  unsigned __int128 M1, M2;
  int x;
  bool lost = false;
  if (d <= 96) {                                  // exact alignment
    M1 = (unsigned __int128)m1 << d;
    M2 = m2;
    x = q.e - 28;
  } else {                                        // operand 2 lies far below
    M1 = (unsigned __int128)m1 << 96;             // the rounding point: keep
    const int sh = d - 96;                        // its floor and a sticky flag
    M2 = sh >= 64 ? 0 : (m2 >> sh);
    lost = sh >= 64 ? m2 != 0 : (m2 & ((((uint64_t)1) << sh) - 1)) != 0;
    x = p.e - 28 - 96;
  }
  if (n1 == n2) return round_general(n1, M1 + M2, x, lost);
  if (M1 == M2 && !lost) return 0u;               // exact cancellation: +0
  if (M1 > M2) return round_general(n1, M1 - M2 - (lost ? 1 : 0), x, lost);
  return round_general(n2, M2 - M1, x, false);     // only reachable with d <= 96
}

__device__ inline win win_of(uint32_t p) { return to_win(decode(p)); }

// ---------------------------------------------------------------------------
// division and square root (long division / digit-by-digit square root, with
// the remainder as the sticky bit)
// ---------------------------------------------------------------------------
__device__ inline uint32_t div_general(dec a, dec b, bool a_nar, bool b_nar) {
  if (a_nar || b_nar || b.s == 0) return kNaR;
  if (a.s == 0) return 0u;
  const bool neg = (a.s < 0) != (b.s < 0);
  const uint64_t ma = (uint64_t)(a.s < 0 ? -(int64_t)a.s : a.s);
  const uint64_t mb = (uint64_t)(b.s < 0 ? -(int64_t)b.s : b.s);
  const uint64_t num = ma << 36;                 // < 2^64
  const uint64_t q = num / mb, r = num % mb;     // q >= 2^35
  return round_general(neg, q, a.sc - b.sc - 36, r != 0);
}

__device__ inline uint32_t sqrt_general(dec a, bool a_nar) {
  if (a_nar || a.s < 0) return kNaR;
  if (a.s == 0) return 0u;
  uint64_t m = (uint64_t)a.s;
  int x = a.sc - 27;                             // a = m * 2^x
  if (x & 1) { m <<= 1; x -= 1; }
  const uint64_t v = m << 34;                    // < 2^63, even shift
  uint64_t r = 0, bit = (uint64_t)1 << 62;
  uint64_t rem = v;
  while (bit > rem) bit >>= 2;
  while (bit) {
    if (rem >= r + bit) { rem -= r + bit; r = (r >> 1) + bit; }
    else { r >>= 1; }
    bit >>= 2;
  }
  return round_general(false, r, x / 2 - 17, rem != 0);
}

// ---------------------------------------------------------------------------
// fast path: multiply and add in window form
// ---------------------------------------------------------------------------

// v_ffbh_i32: position (counted from bit 31) of the first bit that differs
// from the sign bit; -1 for 0 and -1.
__device__ __forceinline__ int ffbh_i32(int32_t x) {
  int r;
  asm("v_ffbh_i32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Round a 64-bit two's-complement value whose leading significant bit is at
// bit 61 to the posit precision of scale sc (fraction length f_s = 27 - (m-1)
// for regime length m, valid for f_s >= 1), returning window form.  The low
// word only matters as a sticky bit, which is folded into bit 0 of the high
// word (the rounding point is at bit >= 2 of the high word, so this is a
// round-to-odd pre-rounding that leaves round-to-nearest-even unchanged).
__device__ __forceinline__ win round_win(uint64_t v, int sc) {
  int32_t h = (int32_t)(v >> 32);
  h |= (uint32_t)v != 0u ? 1 : 0;
  const int t = sc ^ (sc >> 31);                 // |sc| or |sc|-1: regime index
  const int r = 2 + (t >> 2);                    // 29 - f_s
  const int lsb = (h >> (r & 31)) & 1;          // (r is only garbage on lanes
  const int32_t half_m1 = (1 << ((r - 1) & 31)) - 1;   // the caller flags)
  int32_t hr = h + half_m1 + lsb;
  hr &= ~((1 << (r & 31)) - 1);
  win w;
  w.h = hr >> 1;
  w.e = sc;
  return w;
}

// product of decoded operands given as a8 = s_a << 3 and b4 = s_b << 2
__device__ __forceinline__ bool mul_fast(int32_t a8, int32_t sca, int32_t b4, int32_t scb, win& out) {
  const int64_t P = (int64_t)a8 * (int64_t)b4;   // |P| in [2^59, 2^61)
  const int cnt = ffbh_i32((int32_t)(P >> 32));
  const int c2 = cnt - 2;
  const int sc = sca + scb + 4 - cnt;
  const bool ok = ((unsigned)c2 < 30u) & ((unsigned)(sc + 108) < 216u);
  out = round_win((uint64_t)P << (c2 & 63), sc);
  return ok;
}

__device__ __forceinline__ bool add_fast(win a, win b, win& out) {
  const int E = a.e > b.e ? a.e : b.e;
  const int da = min(E - a.e, 63), db = min(E - b.e, 63);
  const int64_t X = ((int64_t)a.h << 32) >> da;
  const int64_t Y = ((int64_t)b.h << 32) >> db;
  const int64_t S = X + Y;                        // |S| <= 2^62
  const int cnt = ffbh_i32((int32_t)(S >> 32));
  const int c2 = cnt - 2;
  const int sc = E + 3 - cnt;
  const bool ok = ((unsigned)c2 < 30u) & ((unsigned)(sc + 108) < 216u);
  out = round_win((uint64_t)S << (c2 & 63), sc);
  return ok;
}

// general product of two decoded operands, in window form
__device__ inline win mul_slow(int32_t a8, int32_t sca, int32_t b4, int32_t scb) {
  dec a, b;
  a.s = a8 >> 3; a.sc = sca;
  b.s = b4 >> 2; b.sc = scb;
  return win_of(mul_general(a, b));
}

__device__ inline win add_slow(win a, win b) { return win_of(add_general(a, b)); }

}  // namespace p32
