// p32_gemm_tile.hpp -- one 64 x 32 tile of the Posit(32,2) Rgemm (and of the
// fused-update chain used by the factorisations), computed by one workgroup of
// 256 threads.  Shared by the Rgemm kernel and the batched factorisation
// kernels.  The blocking, decoding and rounding scheme is described at the top
// of p32_gemm.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "p32_device.hpp"

namespace p32 {

#ifndef P32_GEMM_MIN_WAVES
#define P32_GEMM_MIN_WAVES 4      // minimum waves per SIMD the register budget must allow
#endif

#ifndef P32_GEMM_TM
#define P32_GEMM_TM 4             // rows of C per thread
#endif
#ifndef P32_GEMM_TN
#define P32_GEMM_TN 2             // columns of C per thread
#endif

#ifndef P32_GEMM_UNROLL
#define P32_GEMM_UNROLL 16        // k-steps of a proven k-tile unrolled per loop iteration
#endif
#define P32_STR_(x) #x
#define P32_UNROLL_(n) _Pragma(P32_STR_(unroll n))

#ifndef P32_GEMM_BK
#define P32_GEMM_BK 16            // k-tile depth staged per barrier pair
#endif

// Shape of a workgroup tile: TY x TX threads, each owning a TM x TN
// micro-tile of C, so the workgroup owns BM x BN = (TY TM) x (TX TN)
// outputs; k-tiles of BK.
// PREFETCH: the raw words of the next k-tile are loaded into registers
// before the current k-tile is computed (fewer resident waves have to hide
// the load latency); off for the big tile, whose register budget is spent.
// LATENCY: every k-step on the checked path, whose rounding is computed
// (no table lookup on the accumulator's dependency chain): for launches with
// about one wave per compute unit, where nothing hides that latency.
template <int TM_, int TN_, int TX_, int TY_, bool PREFETCH_, bool LATENCY_ = false>
struct TileShape {
  static constexpr int TM = TM_, TN = TN_, TX = TX_, TY = TY_;
  static constexpr int NT = TX * TY, BM = TY * TM, BN = TX * TN, BK = P32_GEMM_BK;
  static constexpr bool PREFETCH = PREFETCH_, LATENCY = LATENCY_;
};
// 64 x 32 outputs per 256 threads: the Rgemm of large shapes, the batched
// kernels and the factorisations' updates
using BigTile = TileShape<P32_GEMM_TM, P32_GEMM_TN, 16, 16, false>;
// 32 x 32 per 256 threads and 8 x 8 per 64 threads: shapes too small to give
// every compute unit several big tiles
using MidTile = TileShape<2, 2, 16, 16, true>;
using SmallTile = TileShape<1, 1, 8, 8, true>;
using TinyTile = TileShape<1, 1, 8, 8, true, true>;
// 64 x 16 per 256 threads: updates of at most 16 columns (the right-hand
// sides of the batched solves, narrow panel remainders)
using ThinTile = TileShape<4, 1, 16, 16, false>;

constexpr int TM = BigTile::TM, TN = BigTile::TN, NT = BigTile::NT, BK = BigTile::BK;
constexpr int BM = BigTile::BM, BN = BigTile::BN;
constexpr unsigned GROUP_M = 8;             // tile rows per group of the tile order
constexpr int EB = 8192 + 128;           // exponent bias inside the kernel
constexpr int kEZeroB = kEZero + EB;     // biased exponent of zero (> 0)
// Entry i of the rounding table describes scale i - kLutShift.  A sum whose
// aligned exponent is E and whose leading-bit count is cnt has scale
// E + 4 - cnt - EB, i.e. entry (E - cnt) mod 256 since EB = 128 (mod 256);
// a product of staged operands has entry sa + sb + 128 - cnt (see below).
constexpr int kLutShift = 124;

// ---- rare path: exact multiply-add for one element (unbiased interface) ----
static __device__ __noinline__ win madd_slow(win acc, int32_t a8, int32_t sca, int32_t b4, int32_t scb) {
  return add_slow(acc, mul_slow(a8, sca, b4, scb));
}

// epilogue for one element: r = alpha*acc, then r + beta*c (each step on the
// window-form fast path, which falls back to the exact routines; alpha or
// beta equal to one multiplies exactly)
static __device__ __noinline__ uint32_t gemm_epilogue(win acc, int nar, uint32_t alpha, uint32_t beta,
                                               uint32_t c) {
  uint32_t r;
  if (nar || alpha == kNaR) {
    r = kNaR;
  } else {
    const uint32_t a = encode_win(acc);           // acc is exactly a posit
    r = alpha == kOne ? a : encode_win(mul_win(decode(alpha), decode(a)));
  }
  if (beta != 0u) {
    if (r == kNaR || beta == kNaR || c == kNaR) return kNaR;
    const uint32_t t = beta == kOne ? c : encode_win(mul_win(decode(beta), decode(c)));
    r = encode_win(add_win(win_of(r), win_of(t)));
  }
  return r;
}

__device__ __forceinline__ win unbias(win w) {
  win u;
  u.h = w.h;
  u.e = w.h ? w.e - EB : kEZero;
  return u;
}

__device__ __forceinline__ win bias(win u) {
  win w;
  w.h = u.h;
  w.e = u.h ? u.e + EB : kEZeroB;
  return w;
}

// ---- staged operands --------------------------------------------------------
// op(A) element: (s << 3, 16 * (sc + 128)); op(B) element: (s << 2, 16 * sc).
// The scales are kept premultiplied by 16, the size of a rounding-table
// entry, so that a product's table offset is one add and one multiply-add.
__device__ __forceinline__ int2 stage_a(dec d, bool neg) {
  return make_int2((neg ? -d.s : d.s) * 8, 16 * (d.sc + 128));
}
__device__ __forceinline__ int2 stage_b(dec d) { return make_int2(d.s * 4, 16 * d.sc); }
__device__ __forceinline__ int scale_a(int2 a) { return (a.y >> 4) - 128; }
__device__ __forceinline__ int scale_b(int2 b) { return b.y >> 4; }

// ---- checked fast path (any operands; flags what it does not cover) --------
__device__ __forceinline__ bool mul_checked(int2 a, int2 b, win& out) {
  const int64_t P = (int64_t)a.x * (int64_t)b.x;       // |P| in [2^59, 2^61)
  const int cnt = ffbh_i32((int32_t)(P >> 32));
  const int c3 = cnt - 3;
  const int sc = scale_a(a) + scale_b(b) + 4 - cnt;
  out.h = round_h2(fold_sticky((uint64_t)P << (c3 & 63)), sc).h;
  out.e = sc + EB;
  return ((unsigned)c3 < 3u) & scale_ok(sc);
}

__device__ __forceinline__ bool add_checked(win a, win b, win& out) {
  const int E = a.e > b.e ? a.e : b.e;
  const int da = min(E - a.e, 63), db = min(E - b.e, 63);
  const int64_t S = (((int64_t)a.h << 32) >> da) + (((int64_t)b.h << 32) >> db);
  const int cnt = ffbh_i32((int32_t)(S >> 32));
  const int c3 = cnt - 3;
  const int eb = E + 4 - cnt;
  const int sc = eb - EB;
  out.h = round_h2(fold_sticky((uint64_t)S << (c3 & 63)), sc).h;
  out.e = eb;
  return ((unsigned)c3 < 29u) & scale_ok(sc);
}

// ---- unchecked fast path (operands proven in range for the whole k-tile) ---
// Rounding parameters and the result exponent come from the LDS table.  The
// one test left covers cancellation of the sum's high word (c3 < 0) and
// alignments of 64 bits or more, which go to the exact path.
typedef uint4 lut_t;    // x = r, y = 2^(r-1) - 1, z = ~(2^r - 1), w = biased exponent
__device__ __forceinline__ lut_t make_lut_entry(int i) {
  const int sc = i - kLutShift;
  const uint2 p = round_params(sc);
  return make_uint4(p.x & 31u, p.x >> 5, p.y, (uint32_t)(sc + EB));
}
__device__ __forceinline__ const lut_t& lut_at(const lut_t* lut, uint32_t byte_off) {
  return *(const lut_t*)((const char*)lut + byte_off);
}

// x * y + z on the low 24 bits of x and y (one v_mad_i32_i24)
__device__ __forceinline__ int32_t mad_i24(int32_t x, int32_t y, int32_t z) {
  return p32_llvm_mul_i24(x, y) + z;
}

// |x - y| for unsigned x, y (v_sad_u32 with a zero accumulator)
__device__ __forceinline__ uint32_t absdiff(uint32_t x, uint32_t y) {
  uint32_t r;
  asm("v_sad_u32 %0, %1, %2, 0" : "=v"(r) : "v"(x), "v"(y));
  return r;
}

__device__ __forceinline__ win mul_unchecked(int2 a, int2 b, const lut_t* __restrict__ lut) {
  const int64_t P = (int64_t)a.x * (int64_t)b.x;
  const int cnt = ffbh_i32((int32_t)(P >> 32));
  // 16 * (sa + sb + 128 - cnt): entry of scale sa + sb + 4 - cnt
  const lut_t rp = lut_at(lut, (uint32_t)mad_i24(cnt, -16, a.y + b.y));
  const int eb = (int)rp.w;
  win w;
  w.h = round_lut4(fold_sticky((uint64_t)P << ((cnt - 3) & 63)), rp);
  w.e = eb;
  return w;
}

// The operand with the larger exponent is added to the high word of the other
// one shifted right by the exponent difference: the same 64-bit sum as
// aligning both to the larger exponent, with one shift instead of two.
__device__ __forceinline__ win add_unchecked(win a, win b, const lut_t* __restrict__ lut,
                                             uint32_t& badbits) {
  const uint32_t d = absdiff((uint32_t)a.e, (uint32_t)b.e);
  const bool bbig = b.e > a.e;
  const int32_t big = bbig ? b.h : a.h;
  const int32_t small = bbig ? a.h : b.h;
  const int E = bbig ? b.e : a.e;
  const int64_t Y = ((int64_t)small << 32) >> (d & 63);
  const int32_t Shi = (int32_t)(Y >> 32) + big;        // the low word of big << 32 is 0
  const uint64_t S = ((uint64_t)(uint32_t)Shi << 32) | (uint32_t)Y;
  const int cnt = ffbh_i32(Shi);
  const int c3 = cnt - 3;
  badbits |= d | (uint32_t)c3;                          // > 63 means: exact path
  const lut_t rp = lut[(uint32_t)(E - cnt) & 255u];   // entry of scale E + 4 - cnt - EB
  const int eb = (int)rp.w;
  win w;
  w.h = round_lut4(fold_sticky(S << (c3 & 63)), rp);
  w.e = eb;
  return w;
}

// A workgroup-uniform 64-bit value, passed through readfirstlane so that the
// compiler keeps it in scalar registers and does not fold it into per-thread
// addresses that would then stay live across the k loop.
__device__ __forceinline__ int64_t uniform64(int64_t u) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// One k step for the thread's TM x TN accumulators.  Flagged lanes redo the
// whole step on the exact path.
template <bool CHECKED, class S = BigTile>
__device__ __forceinline__ void k_step(win (&acc)[S::TM][S::TN], const int2* __restrict__ Arow,
                                       const int2* __restrict__ Brow, const lut_t* __restrict__ lut,
                                       int tx, int ty) {
  constexpr int TM = S::TM, TN = S::TN;
  int2 a[TM], b[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) a[i] = Arow[ty * TM + i];
#pragma unroll
  for (int j = 0; j < TN; ++j) b[j] = Brow[tx * TN + j];
  win nacc[TM][TN];
  bool bad = false;
  uint32_t badbits = 0;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      if (CHECKED) {
        win pr;
        bad |= !mul_checked(a[i], b[j], pr);
        bad |= !add_checked(acc[i][j], pr, nacc[i][j]);
      } else {
        const win pr = mul_unchecked(a[i], b[j], lut);
        nacc[i][j] = add_unchecked(acc[i][j], pr, lut, badbits);
      }
    }
  if (!CHECKED) bad = badbits > 63u;
  if (bad) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        nacc[i][j] = bias(madd_slow(unbias(acc[i][j]), a[i].x, scale_a(a[i]), b[j].x, scale_b(b[j])));
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = nacc[i][j];
}

// One BM x BN tile of C with origin (i0, j0), computed by the 256 threads of
// the calling workgroup (which must all call it).
// LOWER: only the lower triangle (row >= column) of C is computed and written
// (the trailing update of a Cholesky factorisation).
// CHAIN: instead of Rgemm, each C_ij gets the chain of fused updates
// C_ij = rnd(C_ij - rnd(a_ip * b_pj)) for p = 0, 1, ..., k-1 in order (the
// unblocked factorisations' rank-1 updates, applied k columns at a time); it
// runs as the same k loop with the accumulators starting at C and op(A)
// negated (rnd(-x) = -rnd(x) exactly), and alpha and beta are not used.
// REVK: the k index runs backwards, p = k-1, ..., 0 (the backward
// substitutions of the solves, whose updates come in descending column order).
// LDS of one tile computation; the caller declares it once per kernel
template <class S>
struct TileLdsT {
  int2 As[S::BK][S::BM];   // stage_a of op(A)(i0 + i, p0 + p)
  int2 Bs[S::BK][S::BN];   // stage_b of op(B)(p0 + p, j0 + j)
  lut_t lut[256];          // rounding parameters of scales -124..131
  int rowNaR[S::BM], colNaR[S::BN];
};
using TileLds = TileLdsT<BigTile>;

// UNROLL: k-steps of a proven k-tile unrolled per loop iteration (code size
// against loop overhead; the Rgemm kernel unrolls the whole k-tile).
template <bool TA, bool TB, bool LOWER, bool CHAIN, bool REVK = false, int UNROLL = P32_GEMM_UNROLL,
          class S = BigTile>
__device__ __forceinline__ void gemm_tile(int64_t m, int64_t n, int64_t k, const uint32_t* __restrict__ A,
                                          int64_t lda, const uint32_t* __restrict__ B, int64_t ldb,
                                          uint32_t* __restrict__ C, int64_t ldc, uint32_t alpha,
                                          uint32_t beta, int64_t i0, int64_t j0, TileLdsT<S>& sm) {
  constexpr int TM = S::TM, TN = S::TN, NT = S::NT, BK = S::BK, BM = S::BM, BN = S::BN;
  auto& As = sm.As;
  auto& Bs = sm.Bs;
  auto& lut = sm.lut;
  auto& rowNaR = sm.rowNaR;
  auto& colNaR = sm.colNaR;

  const int tid = threadIdx.x;
  const int tx = tid % S::TX, ty = tid / S::TX;
  if (LOWER && i0 + BM - 1 < j0) return;          // tile entirely above the diagonal
  __syncthreads();                                // LDS of a previous tile no longer in use
  if (tid < BM) rowNaR[tid] = 0;
  if (tid < BN) colNaR[tid] = 0;
  static_assert(256 % NT == 0, "table fill");
#pragma unroll
  for (int e = 0; e < 256; e += NT) lut[e + tid] = make_lut_entry(e + tid);

  win acc[TM][TN];
  uint32_t cnar = 0;            // CHAIN: bit i*TN+j set when C_ij starts as NaR
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j].h = 0;
      acc[i][j].e = kEZeroB;
      if (CHAIN) {
        const int64_t gi = i0 + ty * TM + i, gj = j0 + tx * TN + j;
        if (gi < m && gj < n && !(LOWER && gj > gi)) {
          const uint32_t c = C[gi * ldc + gj];
          if (c == kNaR) cnar |= 1u << (i * TN + j);
          else acc[i][j] = bias(win_of(c));
        }
      }
    }

  // Staging addresses.  Element l of this thread's share of a k-tile sits at
  // a workgroup-uniform offset (a function of l and p0, kept in scalar
  // registers) plus a per-thread offset that is the same for every l and
  // every k-tile, so the k loop carries one 64-bit offset per operand
  // instead of one pointer per staged element.
  static_assert(NT % BK == 0 && NT % BM == 0 && NT % BN == 0, "staging layout");
  const int a_r = TA ? tid / BM : tid / BK;     // stored row of A within the l-group
  const int a_c = TA ? tid % BM : tid % BK;     // stored column
  const int b_r = TB ? tid / BK : tid / BN;
  const int b_c = TB ? tid % BK : tid % BN;
  const int64_t a_off = (int64_t)a_r * lda + a_c;
  const int64_t b_off = (int64_t)b_r * ldb + b_c;

  // rows of op(A) and columns of op(B) left in this tile (clamped: a tile
  // index is below 64), compared with 32-bit per-thread indices
  const int rem_m = (int)min(m - i0, (int64_t)BM), rem_n = (int)min(n - j0, (int64_t)BN);

  // PREFETCH: raw words of this thread's share of the next k-tile
  constexpr int LA = (BM * BK) / NT, LB = (BN * BK) / NT;
  uint32_t ra[S::PREFETCH ? LA : 1], rb[S::PREFETCH ? LB : 1];
  // op(A)(i0 + ii, p0 + pp) and op(B)(p0 + pp, j0 + jj) for element l:
  // 0 beyond k, 1.0 beyond m or n (results discarded)
  auto fetch_a = [&](int64_t q0, int l) -> uint32_t {
    const int ii = TA ? a_c : a_r + l * (NT / BK);
    const int pp = TA ? a_r + l * (NT / BM) : a_c;
    if (q0 + pp >= k) return 0u;
    if (ii >= rem_m) return kOne;
    if (REVK) {
      const int64_t gi = i0 + ii, gk = k - 1 - (q0 + pp);
      return TA ? A[gk * lda + gi] : A[gi * lda + gk];
    }
    const int64_t u = TA ? (q0 + l * (NT / BM)) * lda + i0 : (i0 + l * (NT / BK)) * lda + q0;
    return A[uniform64(u) + a_off];
  };
  auto fetch_b = [&](int64_t q0, int l) -> uint32_t {
    const int jj = TB ? b_r + l * (NT / BK) : b_c;
    const int pp = TB ? b_c : b_r + l * (NT / BN);
    if (q0 + pp >= k) return 0u;
    if (jj >= rem_n) return kOne;
    if (REVK) {
      const int64_t gj = j0 + jj, gk = k - 1 - (q0 + pp);
      return TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
    }
    const int64_t u = TB ? (j0 + l * (NT / BK)) * ldb + q0 : (q0 + l * (NT / BN)) * ldb + j0;
    return B[uniform64(u) + b_off];
  };
  if constexpr (S::PREFETCH) {
#pragma unroll
    for (int l = 0; l < LA; ++l) ra[l] = fetch_a(0, l);
#pragma unroll
    for (int l = 0; l < LB; ++l) rb[l] = fetch_b(0, l);
  }

  for (int64_t p0 = 0; p0 < k; p0 += BK) {
    int my_ok = 1;
    const int rem_k = (int)min(k - p0, (int64_t)BK);
    __syncthreads();
    if constexpr (S::PREFETCH) {
#pragma unroll
      for (int l = 0; l < LA; ++l) {
        const int ii = TA ? a_c : a_r + l * (NT / BK);
        const int pp = TA ? a_r + l * (NT / BM) : a_c;
        uint32_t v = ra[l];
        if (v == kNaR) { rowNaR[ii] = 1; v = kOne; }
        const dec d = decode(v);
        my_ok &= (d.s != 0) & ((unsigned)(d.sc + 53) <= 102u);
        As[pp][ii] = stage_a(d, CHAIN);
      }
#pragma unroll
      for (int l = 0; l < LB; ++l) {
        const int jj = TB ? b_r + l * (NT / BK) : b_c;
        const int pp = TB ? b_c : b_r + l * (NT / BN);
        uint32_t v = rb[l];
        if (v == kNaR) { colNaR[jj] = 1; v = kOne; }
        const dec d = decode(v);
        my_ok &= (d.s != 0) & ((unsigned)(d.sc + 53) <= 102u);
        Bs[pp][jj] = stage_b(d);
      }
      if (p0 + BK < k) {
#pragma unroll
        for (int l = 0; l < LA; ++l) ra[l] = fetch_a(p0 + BK, l);
#pragma unroll
        for (int l = 0; l < LB; ++l) rb[l] = fetch_b(p0 + BK, l);
      }
    } else {
#pragma unroll
    for (int l = 0; l < (BM * BK) / NT; ++l) {
      // op(A)(i0 + ii, p0 + pp) with ii, pp this thread's element l
      const int ii = TA ? a_c : a_r + l * (NT / BK);
      const int pp = TA ? a_r + l * (NT / BM) : a_c;
      uint32_t v;
      if (pp >= rem_k) v = 0u;
      else if (ii >= rem_m) v = kOne;
      else if (REVK) {
        const int64_t gi = i0 + ii, gk = k - 1 - (p0 + pp);
        v = TA ? A[gk * lda + gi] : A[gi * lda + gk];
      }
      else {
        const int64_t u = TA ? (p0 + l * (NT / BM)) * lda + i0 : (i0 + l * (NT / BK)) * lda + p0;
        v = A[uniform64(u) + a_off];
      }
      if (v == kNaR) { rowNaR[ii] = 1; v = kOne; }
      const dec d = decode(v);
      my_ok &= (d.s != 0) & ((unsigned)(d.sc + 53) <= 102u);
      As[pp][ii] = stage_a(d, CHAIN);
    }
#pragma unroll
    for (int l = 0; l < (BN * BK) / NT; ++l) {
      // op(B)(p0 + pp, j0 + jj)
      const int jj = TB ? b_r + l * (NT / BK) : b_c;
      const int pp = TB ? b_c : b_r + l * (NT / BN);
      uint32_t v;
      if (pp >= rem_k) v = 0u;
      else if (jj >= rem_n) v = kOne;
      else if (REVK) {
        const int64_t gj = j0 + jj, gk = k - 1 - (p0 + pp);
        v = TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
      }
      else {
        const int64_t u = TB ? (j0 + l * (NT / BK)) * ldb + p0 : (p0 + l * (NT / BN)) * ldb + j0;
        v = B[uniform64(u) + b_off];
      }
      if (v == kNaR) { colNaR[jj] = 1; v = kOne; }
      const dec d = decode(v);
      my_ok &= (d.s != 0) & ((unsigned)(d.sc + 53) <= 102u);
      Bs[pp][jj] = stage_b(d);
    }
    }
    // Block-uniform choice of the inner loop for this k-tile.  The unchecked
    // loop is exact when every staged operand is nonzero with scale in
    // [-53, 49] (products then have scales in [-106, 99]) and every
    // accumulator is zero or has scale in [-106, 100].  Sums then keep
    // scales in [-108, 104], inside the fast range: with |p| >= 2^-106, a
    // sum acc + p either has |acc| < |p|/2 and so |sum| > 2^-107, or both
    // terms are multiples of 2^-108 and a nonzero sum is >= 2^-108; and 16
    // products below 2^100 cannot lift |acc| < 2^101 past 2^105.  Left to
    // test: cancellation to zero or by more than 28 bits, and alignment
    // shifts of 64 bits or more (e.g. a zero accumulator).
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        my_ok &= (acc[i][j].h == 0) | ((unsigned)(acc[i][j].e - EB + 106) <= 206u);
    const bool safe = __syncthreads_and(my_ok);

    if constexpr (S::LATENCY) {
      P32_UNROLL_(UNROLL)
      for (int p = 0; p < BK; ++p) k_step<true, S>(acc, As[p], Bs[p], lut, tx, ty);
    } else if (p0 == 0) {  // first step: accumulators not yet tested, use the checked path
      k_step<true, S>(acc, As[0], Bs[0], lut, tx, ty);
      if (safe) {
#pragma unroll 1
        for (int p = 1; p < BK; ++p) k_step<false, S>(acc, As[p], Bs[p], lut, tx, ty);
      } else {
#pragma unroll 1
        for (int p = 1; p < BK; ++p) k_step<true, S>(acc, As[p], Bs[p], lut, tx, ty);
      }
    } else if (safe) {
      P32_UNROLL_(UNROLL)
      for (int p = 0; p < BK; ++p) k_step<false, S>(acc, As[p], Bs[p], lut, tx, ty);
    } else {
#pragma unroll 1
      for (int p = 0; p < BK; ++p) k_step<true, S>(acc, As[p], Bs[p], lut, tx, ty);
    }
  }
  __syncthreads();

#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int64_t gi = i0 + ty * TM + i;
    if (gi >= m) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t gj = j0 + tx * TN + j;
      if (gj >= n || (LOWER && gj > gi)) continue;
      const int nar = rowNaR[ty * TM + i] | colNaR[tx * TN + j];
      if (CHAIN) {
        C[gi * ldc + gj] = nar || ((cnar >> (i * TN + j)) & 1u) ? kNaR : encode_exact(unbias(acc[i][j]));
        continue;
      }
      const uint32_t c = beta ? C[gi * ldc + gj] : 0u;
      C[gi * ldc + gj] = gemm_epilogue(unbias(acc[i][j]), nar, alpha, beta, c);
    }
  }
}


// XCD-aware tile order.  The dispatcher places workgroup g on XCD g % 8, and
// each XCD has its own L2, so consecutive tiles are handed to the same XCD:
// XCD x takes the x-th eighth of the tile sequence.  The sequence walks groups
// of GROUP_M tile rows column by column, so the tiles that are resident on an
// XCD at one time form a compact block of C and share their A and B panels in
// that XCD's L2.
template <class S = BigTile>
__device__ __forceinline__ void tile_origin(int64_t m, int64_t n, unsigned g, int64_t& i0, int64_t& j0) {
  constexpr int BM = S::BM, BN = S::BN;
  const unsigned nrow = (unsigned)((m + BM - 1) / BM), ncol = (unsigned)((n + BN - 1) / BN);
  const unsigned G = nrow * ncol;
  if (G % 8u == 0u) g = (g % 8u) * (G / 8u) + g / 8u;
  const unsigned per_group = GROUP_M * ncol;
  const unsigned first_row = (g / per_group) * GROUP_M;
  const unsigned rows_here = min(nrow - first_row, (unsigned)GROUP_M);
  const unsigned in_group = g % per_group;
  i0 = (int64_t)(first_row + in_group % rows_here) * BM;
  j0 = (int64_t)(in_group / rows_here) * BN;
}

}  // namespace p32
