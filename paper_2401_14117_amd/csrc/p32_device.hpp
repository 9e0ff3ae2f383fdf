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
//    |h| <= 2^28 and an exponent e, x = h * 2^(e - 27).  Rounded values keep
//    their significand bits at h[27..0]; e is the scale (one less for the
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
  int32_t h;    // |h| <= 2^28
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
  w.h = d.s;
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

// round_general for an exact value whose integer part M fits in 64 bits
__device__ inline uint32_t round_general64(bool neg, uint64_t M, int x, bool sticky) {
  if (M == 0) {
    if (!sticky) return 0u;
    return neg ? 0xFFFFFFFFu : 1u;
  }
  const int t = 63 - __clzll(M);
  const int sc = x + t;
  uint32_t P;
  const bool pow2 = (M & (M - 1)) == 0 && !sticky;
  if (sc >= kMaxScale) {
    P = kMaxpos;
  } else if (sc < -kMaxScale || (sc == -kMaxScale && pow2)) {
    P = 1u;
  } else {
    const int k = sc >> 2;
    const int e = sc & 3;
    const int R = k >= 0 ? k + 2 : 1 - k;
    const uint64_t regime = k >= 0 ? ((((uint64_t)1 << (k + 1)) - 1) << 1) : (uint64_t)1;
    const uint64_t f64 = t == 0 ? 0 : (M << (64 - t));   // fraction bits, left-aligned
    const int fsh = R + 2;
    bool s = sticky || (f64 & ((((uint64_t)1) << fsh) - 1)) != 0;
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
  return round_general64(neg, ma * mb, a.sc + b.sc - 54, false);
}

// pattern of a window-form value that is exactly representable
__device__ inline uint32_t encode_exact(win a) {
  if (a.h == 0) return 0u;
  const bool neg = a.h < 0;
  const uint64_t m = (uint64_t)(neg ? -(int64_t)a.h : a.h);
  return round_general64(neg, m, a.e - 27, false);
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
    x = q.e - 27;
  } else {                                        // operand 2 lies far below
    M1 = (unsigned __int128)m1 << 96;             // the rounding point: keep
    const int sh = d - 96;                        // its floor and a sticky flag
    M2 = sh >= 64 ? 0 : (m2 >> sh);
    lost = sh >= 64 ? m2 != 0 : (m2 & ((((uint64_t)1) << sh) - 1)) != 0;
    x = p.e - 27 - 96;
  }
  if (n1 == n2) return round_general(n1, M1 + M2, x, lost);
  if (M1 == M2 && !lost) return 0u;               // exact cancellation: +0
  if (M1 > M2) return round_general(n1, M1 - M2 - (lost ? 1 : 0), x, lost);
  return round_general(n2, M2 - M1, x, false);     // only reachable with d <= 96
}

__device__ inline win win_of(uint32_t p) { return to_win(decode(p)); }

// ---------------------------------------------------------------------------
// division and square root: exact integer quotient / integer square root
// (from a binary64 estimate corrected in integers), the remainder as sticky
// ---------------------------------------------------------------------------
__device__ inline uint32_t div_general(dec a, dec b, bool a_nar, bool b_nar) {
  if (a_nar || b_nar || b.s == 0) return kNaR;
  if (a.s == 0) return 0u;
  const bool neg = (a.s < 0) != (b.s < 0);
  const uint64_t ma = (uint64_t)(a.s < 0 ? -(int64_t)a.s : a.s);
  const uint64_t mb = (uint64_t)(b.s < 0 ? -(int64_t)b.s : b.s);
  const uint64_t num = ma << 36;                 // < 2^64, exact in binary64
  // Quotient estimate from a binary64 division (within 2^-16 of num/mb,
  // which is below 2^37), then the exact floor and remainder in integers.
  uint64_t q = (uint64_t)((double)num / (double)mb);
  int64_t r = (int64_t)(num - q * mb);           // |r| < 2 mb
  if (r < 0) { q -= 1; r += (int64_t)mb; }
  else if (r >= (int64_t)mb) { q += 1; r -= (int64_t)mb; }
  return round_general64(neg, q, a.sc - b.sc - 36, r != 0);
}

__device__ inline uint32_t sqrt_general(dec a, bool a_nar) {
  if (a_nar || a.s < 0) return kNaR;
  if (a.s == 0) return 0u;
  uint64_t m = (uint64_t)a.s;
  int x = a.sc - 27;                             // a = m * 2^x
  if (x & 1) { m <<= 1; x -= 1; }
  const uint64_t v = m << 34;                    // < 2^63, at most 29 significant bits
  // integer square root: binary64 estimate (within one unit), then exact fix-up
  uint64_t r = (uint64_t)sqrt((double)v);
  if (r * r > v) r -= 1;
  else if ((r + 1) * (r + 1) <= v) r += 1;
  return round_general64(false, r, x / 2 - 17, v != r * r);
}

// ---------------------------------------------------------------------------
// fast path: multiply and add in window form
// ---------------------------------------------------------------------------

// LLVM's AMDGPU intrinsics for v_ffbh_i32 and v_mul_i32_i24, called directly
// (no clang builtin exposes them); unlike inline asm they leave the
// instruction scheduler and the hazard recognizer full knowledge.
extern "C" __device__ __attribute__((const)) int p32_llvm_sffbh(int) __asm("llvm.amdgcn.sffbh.i32");
extern "C" __device__ __attribute__((const)) int p32_llvm_mul_i24(int, int) __asm("llvm.amdgcn.mul.i24");

// v_ffbh_i32: position (counted from bit 31) of the first bit that differs
// from the sign bit; -1 for 0 and -1.
__device__ __forceinline__ int ffbh_i32(int32_t x) { return p32_llvm_sffbh(x); }

__device__ __forceinline__ uint32_t bfm(int width) {   // (1 << width) - 1
  uint32_t r;
  asm("v_bfm_b32 %0, %1, 0" : "=v"(r) : "v"(width));
  return r;
}

// Fold the low word of a 64-bit value into the high word as a sticky bit:
// returns 2*hi + (lo != 0), a round-to-odd pre-rounding one bit below hi.
__device__ __forceinline__ int32_t fold_sticky(uint64_t v) {
  const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
  uint32_t r;
  uint64_t carry;   // lane mask (lo != 0), fed back as the carry-in
  asm("v_cmp_ne_u32_e64 %1, 0, %2\n\tv_addc_co_u32_e64 %0, %1, %3, %3, %1"
      : "=v"(r), "=&s"(carry) : "v"(lo), "v"(hi));
  return (int32_t)r;
}

// Round h2 (leading significant bit at bit 29, sticky in bit 0) to the posit
// precision of scale sc: f_s = 27 - s fraction bits with s = m - 1 the regime
// index, valid for f_s >= 1.  The kept bits are h2[29 .. s+2]; the guard bit
// is h2[s+1], so bit 0 is always below it and the round-to-odd sticky leaves
// round-to-nearest-even unchanged.  Returns window form (leading bit at 27).
__device__ __forceinline__ win round_h2(int32_t h2, int sc) {
  const int t = sc ^ (sc >> 31);                 // sc >= 0 ? sc : -sc - 1
  const int s = t >> 2;                          // regime index m - 1
  const int r = s + 2;                           // rounding position
  const int32_t half_m1 = (int32_t)bfm(s + 1);   // 2^(r-1) - 1
  const int32_t lsb = (int32_t)__builtin_amdgcn_ubfe((uint32_t)h2, (uint32_t)r, 1u);
  const int32_t q = (h2 + half_m1 + lsb) >> r;   // nearest, ties to even
  win w;
  w.h = q << s;
  w.e = sc;
  return w;
}

// Rounding parameters of one scale, packed for round_lut:
//   x = (2^(r-1) - 1) << 5 | r   (r = s + 2 in the low five bits, where the
//                                  shift and bit-field instructions read it)
//   y = ~(2^r - 1)               (clears the bits below the rounding point)
__device__ __forceinline__ uint2 round_params(int sc) {
  const int t = sc ^ (sc >> 31);
  int s = t >> 2;
  if (s > 26) s = 26;                            // f_s = 0 or tapered: unused
  const int r = s + 2;
  uint2 p;
  p.x = (((1u << (r - 1)) - 1u) << 5) | (uint32_t)r;
  p.y = ~((1u << r) - 1u);
  return p;
}

// round_h2 with the scale-dependent parameters taken from a table entry
__device__ __forceinline__ int32_t round_lut(int32_t h2, uint2 p) {
  const int32_t lsb = (int32_t)__builtin_amdgcn_ubfe((uint32_t)h2, p.x, 1u);
  const int32_t q = h2 + (int32_t)(p.x >> 5) + lsb;
  return (q & (int32_t)p.y) >> 2;
}

// The same parameters unpacked into one 16-byte entry: x = r, y = 2^(r-1) - 1,
// z = ~(2^r - 1), so no shift is needed to separate them.
__device__ __forceinline__ uint4 round_params4(int sc) {
  const uint2 p = round_params(sc);
  return make_uint4(p.x & 31u, p.x >> 5, p.y, 0u);
}

__device__ __forceinline__ int32_t round_lut4(int32_t h2, uint4 p) {
  const int32_t lsb = (int32_t)__builtin_amdgcn_ubfe((uint32_t)h2, p.x, 1u);
  const int32_t q = h2 + (int32_t)p.y + lsb;
  return (q & (int32_t)p.z) >> 2;
}

// product of decoded operands given as a8 = s_a << 3 and b4 = s_b << 2:
// |P| in [2^59, 2^61), normalised to a leading bit at 60.
__device__ __forceinline__ win mul_core(int32_t a8, int32_t sca, int32_t b4, int32_t scb, int& c3) {
  const int64_t P = (int64_t)a8 * (int64_t)b4;
  const int cnt = ffbh_i32((int32_t)(P >> 32));
  c3 = cnt - 3;
  const int sc = sca + scb + 4 - cnt;
  return round_h2(fold_sticky((uint64_t)P << (c3 & 63)), sc);
}

// sum of two window-form values: both are aligned to the larger exponent
// (bit 59 <-> 2^E) in 64-bit two's complement, so |S| <= 2^61.  An operand
// shifted past bit 0 only loses bits far below the rounding point (it then
// sits >= 33 bits below the other one, whose last bit is at >= 32), where the
// truncation toward -inf cannot cross a rounding boundary.
__device__ __forceinline__ win add_core(win a, win b, int& c3) {
  const int E = a.e > b.e ? a.e : b.e;
  const int da = min(E - a.e, 63), db = min(E - b.e, 63);
  const int64_t X = ((int64_t)a.h << 32) >> da;
  const int64_t Y = ((int64_t)b.h << 32) >> db;
  const int64_t S = X + Y;
  const int cnt = ffbh_i32((int32_t)(S >> 32));
  c3 = cnt - 3;                                  // valid when 0 <= c3 < 29
  const int sc = E + 4 - cnt;
  return round_h2(fold_sticky((uint64_t)S << (c3 & 63)), sc);
}

// fast-range test of a result scale: f_s >= 1 and outside the tapered regime
__device__ __forceinline__ bool scale_ok(int sc) { return (unsigned)(sc + 108) < 216u; }

// checked forms: return false when the lane must take the exact rare path
__device__ __forceinline__ bool mul_fast(int32_t a8, int32_t sca, int32_t b4, int32_t scb, win& out) {
  int c3;
  out = mul_core(a8, sca, b4, scb, c3);
  return ((unsigned)c3 < 3u) & scale_ok(out.e);
}

__device__ __forceinline__ bool add_fast(win a, win b, win& out) {
  int c3;
  out = add_core(a, b, c3);
  return ((unsigned)c3 < 29u) & scale_ok(out.e);
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

namespace p32 {

// ---------------------------------------------------------------------------
// pattern-level operations for the factorisation and solve kernels
// ---------------------------------------------------------------------------

// Pattern of an exactly representable window-form value.  Scales with f_s >= 1
// are encoded directly (regime run, terminator, two exponent bits, the top f_s
// fraction bits); others go through the general rounding.
__device__ inline uint32_t encode_win(win w) {
  if (w.h == 0) return 0u;
  const bool neg = w.h < 0;
  uint32_t mag = (uint32_t)(neg ? -w.h : w.h);
  int sc = w.e;
  if (mag >= (1u << 28)) { mag >>= 1; sc += 1; }   // 2^(e+1) held as 2^28
  if (!scale_ok(sc)) return encode_exact(w);
  const int k = sc >> 2, e = sc & 3;
  const int R = k >= 0 ? k + 2 : 1 - k;           // run + terminator
  const uint32_t regime = k >= 0 ? (0x7FFFFFFFu >> (30 - k)) << (30 - k) : (1u << (30 + k));
  const uint32_t frac = mag - (1u << 27);
  const uint32_t p = regime | ((uint32_t)e << (29 - R)) | (frac >> (R - 2));
  return neg ? 0u - p : p;
}

// decoded form of a window-form value (exactly a posit): |s| in [2^27, 2^28)
__device__ __forceinline__ dec dec_of_win(win w) {
  dec d;
  const bool big = w.h >= (1 << 28) || w.h <= -(1 << 28);   // a power of two held one bit high
  d.s = big ? (w.h >> 1) : w.h;
  d.sc = w.h == 0 ? kEZero : (big ? w.e + 1 : w.e);
  return d;
}

// rnd(a / b) in window form for decoded a, b (b nonzero, neither NaR), with
// rcp_b = 1.0 / |b.s| computed beforehand (a divisor reused along a chain
// costs one binary64 multiply per quotient).  Everything stays in binary64:
// floor(num * rcp_b) is within one unit of the 37-bit integer quotient
// q = floor(num / |b.s|), num = |a.s| 2^36; the remainder num - q |b.s| is
// exact in one fused multiply-add (it is an integer below 2^30), which fixes
// q up and gives the sticky bit; q, an integer below 2^37, is then read from
// the bits of its binary64 representation.
__device__ __forceinline__ void div_quotient(dec a, dec b, double rcp_b, uint32_t& hi, uint32_t& lo,
                                             bool& rem) {
  const double ma = (double)(a.s < 0 ? -a.s : a.s);
  const double mb = (double)(b.s < 0 ? -b.s : b.s);
  const double num = ma * 68719476736.0;          // |a.s| 2^36, exact
  double q = floor(num * rcp_b);
  double r = fma(-q, mb, num);                    // exact, |r| < 2 |b.s|
  const double adj = r < 0.0 ? -1.0 : (r >= mb ? 1.0 : 0.0);
  q += adj;
  r = fma(-adj, mb, r);
  // q in [2^35, 2^37): significand bits [51:0] of q hold q below its leading bit
  const uint64_t bits = (uint64_t)__double_as_longlong(q);
  hi = (uint32_t)(bits >> 32);
  lo = (uint32_t)bits;
  rem = r != 0.0;
}

// the quotient rounded at a scale sc inside the fast range: the top 30 bits
// of the significand (leading bit at 29), the rest of it and the remainder
// folded into bit 0
__device__ __forceinline__ win div_round_fast(bool neg, uint32_t hi, uint32_t lo, bool rem, int sc) {
  const uint32_t top = ((hi & 0xFFFFFu) | 0x100000u) << 9 | (lo >> 23);
  const int32_t h2 = (int32_t)((top & ~1u) | (uint32_t)(((lo & 0xFFFFFFu) != 0u) | rem));
  return round_h2(neg ? -h2 : h2, sc);            // round to nearest even is odd-symmetric
}

__device__ inline win div_win(dec a, dec b, double rcp_b) {
  win w;
  if (a.s == 0) {
    w.h = 0;
    w.e = kEZero;
    return w;
  }
  const bool neg = (a.s < 0) != (b.s < 0);
  uint32_t hi, lo;
  bool rem;
  div_quotient(a, b, rcp_b, hi, lo, rem);
  const int L = (int)(hi >> 20) - 1023;           // 35 or 36
  const int sc = a.sc - b.sc - 36 + L;
  if (scale_ok(sc)) return div_round_fast(neg, hi, lo, rem, sc);
  const uint64_t qi = ((((uint64_t)(hi & 0xFFFFFu) | 0x100000u) << 32) | lo) >> (52 - L);
  return win_of(round_general64(neg, qi, a.sc - b.sc - 36, rem));
}

// div_win without branches, for chains where one lane's quotient is needed
// by the whole wave: ok is false when div_win must be called instead (a zero
// dividend, or a quotient scale outside the fast range); the returned value
// is then meaningless.  b must be nonzero.
__device__ __forceinline__ win div_win_fast(dec a, dec b, double rcp_b, bool& ok) {
  uint32_t hi, lo;
  bool rem;
  div_quotient(a, b, rcp_b, hi, lo, rem);
  const int sc = a.sc - b.sc - 36 + (int)(hi >> 20) - 1023;
  ok = (a.s != 0) & scale_ok(sc);
  return div_round_fast((a.s < 0) != (b.s < 0), hi, lo, rem, sc);
}

// rnd(sqrt(a)) in window form for a decoded a > 0.  With a = m 2^x, x even,
// v = m 2^34 (at most 29 significant bits, exact in binary64) and r =
// floor(sqrt(v)): the binary64 square root is within one unit of r, and
// r^2 - v, an integer below 2^34 in magnitude, is exact in one fused
// multiply-add, which fixes r up and gives the sticky bit.  sqrt(a) =
// (r + f) 2^(x/2 - 17) with 0 <= f < 1; its scale is inside the fast range.
__device__ inline win sqrt_win(dec a) {
  int x = a.sc - 27;                              // a = a.s 2^x
  double m = (double)a.s;
  if (x & 1) {
    m *= 2.0;
    x -= 1;
  }
  const double v = m * 17179869184.0;             // m 2^34, exact
  double r = floor(sqrt(v));
  double d = fma(r, r, -v);                       // r^2 - v, exact
  if (d > 0.0) {
    d -= 2.0 * r - 1.0;
    r -= 1.0;
  } else if (d + 2.0 * r + 1.0 <= 0.0) {
    d += 2.0 * r + 1.0;
    r += 1.0;
  }
  const uint32_t ri = (uint32_t)r;                // in [2^30, 2^32)
  const int L = 31 - __clz(ri);                   // 30 or 31
  const int sh = L - 28;                          // 2 or 3
  const uint32_t kept = ri >> sh;                 // leading bit at 28
  const uint32_t lost = ri & ((1u << sh) - 1u);
  const int32_t h2 = (int32_t)(2u * kept + (uint32_t)((lost != 0u) | (d != 0.0)));
  return round_h2(h2, x / 2 - 17 + L);
}

// A divisor prepared once for many quotients: decoded, with its binary64
// reciprocal; NaR and zero divisors give NaR quotients.
struct divisor {
  dec d;
  double rcp;
  bool bad;
};

__device__ __forceinline__ divisor make_divisor(uint32_t b) {
  divisor v;
  v.d = decode(b);
  v.bad = b == kNaR || v.d.s == 0;
  v.rcp = v.bad ? 0.0 : 1.0 / (double)(v.d.s < 0 ? -(int64_t)v.d.s : (int64_t)v.d.s);
  return v;
}

// rnd(a / b) on patterns with b prepared by make_divisor
__device__ __forceinline__ uint32_t p_div_by(uint32_t a, const divisor& b) {
  if (a == kNaR || b.bad) return kNaR;
  return encode_win(div_win(decode(a), b.d, b.rcp));
}

// rnd(x * y) in window form, fast path with exact fallback
__device__ inline win mul_win(dec x, dec y) {
  win r;
  if (x.s != 0 && y.s != 0 && mul_fast(x.s * 8, x.sc, y.s * 4, y.sc, r)) return r;
  return win_of(mul_general(x, y));
}

// rnd(a + b) of two window-form values, fast path with exact fallback
__device__ inline win add_win(win a, win b) {
  win r;
  if (add_fast(a, b, r)) return r;
  return win_of(add_general(a, b));
}

// acc - rnd(b * c) rounded, with acc in window form (exactly a posit value)
// and b, c decoded, none of them NaR: a running value kept decoded across a
// chain of fused updates, encoded only when it is published
__device__ inline win fms_win(win acc, dec b, dec c) {
  win pr = mul_win(b, c);
  pr.h = -pr.h;
  return add_win(acc, pr);
}

// rnd(a - rnd(b * c)), with b and c given as patterns and already decoded
__device__ inline uint32_t p_fms_pre(uint32_t a, uint32_t b, dec db, uint32_t c, dec dc) {
  if (a == kNaR || b == kNaR || c == kNaR) return kNaR;
  win pr = mul_win(db, dc);
  pr.h = -pr.h;
  return encode_win(add_win(win_of(a), pr));
}

// rnd(a - rnd(b * c)) on patterns
__device__ inline uint32_t p_fms(uint32_t a, uint32_t b, uint32_t c) {
  return p_fms_pre(a, b, decode(b), c, decode(c));
}

__device__ inline uint32_t p_div(uint32_t a, uint32_t b) {
  return div_general(decode(a), decode(b), a == kNaR, b == kNaR);
}

__device__ inline uint32_t p_sqrt(uint32_t a) {
  if (a == kNaR || (int32_t)a < 0) return kNaR;
  if (a == 0u) return 0u;
  return encode_win(sqrt_win(decode(a)));
}

// key of |x| for pivot search: posit order is signed-integer order of the
// patterns and |NaR| = NaR is the smallest; ties prefer the smaller row
__device__ __forceinline__ unsigned long long pivot_key(uint32_t x, int64_t row) {
  const int32_t s = (int32_t)x;
  const int32_t a = x == kNaR ? INT32_MIN : (s < 0 ? -s : s);
  return ((unsigned long long)((uint32_t)a ^ 0x80000000u) << 32) |
         (unsigned long long)(0xFFFFFFFFu - (uint32_t)row);
}

}  // namespace p32
