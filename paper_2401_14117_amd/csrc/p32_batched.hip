// p32_batched.hip -- variable-size batched Posit(32,2) LU and Cholesky
// factorisations and solves: many small independent systems (the sizes of the
// paper's LU and Cholesky study, Section 5, in large numbers) in one launch.
//
// Workgroup g (256 threads) runs the whole factorisation (and solve) of
// system g.  The dispatcher starts workgroups in index order as earlier ones
// retire, so a batch sorted by decreasing size is scheduled largest first
// onto whichever compute unit frees up, and the launch needs no counter,
// workspace or memset (it can be captured in a graph as is).
//
// Every matrix is processed in the schedule of the single-matrix routines
// with the same block size nb, so the results are bit-identical to them:
//
//  LU, per panel [j, j+jb): sub-panels of `sub` columns [c0, c0+w):
//    (i)   unblocked LU of the sub-panel on rows [c0, n) (pivot search,
//          swap inside the sub-panel, scaling, rank-1 updates);
//    (ii)  the sub-panel's interchanges applied to all other columns;
//    (iii) its unit-lower triangle applied to rows [c0, c0+w) of the panel
//          columns right of it (column by column, ascending);
//    (iv)  fused-update chain over the sub-panel's columns for all rows below
//          it, on the panel columns right of it;
//    then, with all of the panel's interchanges in place, U12 = L11^-1 A12
//    with the same sub-panels ((iii) on the columns right of the panel, then
//    the chain for the panel rows below the sub-panel), and the trailing
//    update Rgemm(-1, 1, L21, U12) with k = jb.
//  Each element thus receives the unblocked order's updates in the same
//  sequence (the interchanges only move whole rows).
//
//  Cholesky, per diagonal block [j, j+jb): sub-blocks [c0, c0+w):
//    unblocked Cholesky of the w x w sub-block; the block's rows below it
//    solved against it column by column (divide, then update the sub-block's
//    later columns); fused-update chain over its columns for the rest of the
//    block's lower triangle.  If a diagonal fails at column c, the rows below
//    the sub-block get the column steps before c and the rest of the block
//    the chain over [c0, c): exactly the state the unblocked order leaves.
//    Then L21 with the same sub-blocks, and the lower triangle of
//    Rgemm(-1, 1, L21, L21^T).
//
//  Solves: the row interchanges (LU), then forward and backward substitution
//  in blocks of 64 rows: the diagonal block column by column (one wave per
//  right-hand side, one row per lane), then one fused-update chain over the
//  block's columns for all rows beyond it (in descending column order for
//  the backward pass).
//
// The sub-panel width `sub` only regroups the work: every element still gets
// its updates in the unblocked order, so any width gives the same bits.  It
// is chosen per system from a table of size buckets (the autotuner measures
// the fastest width of each bucket on the device): narrow sub-panels put more
// of a large matrix's updates on the tile routine, and a width of at least n
// factors a small matrix unblocked, with no tile overhead at all.
#include <hip/hip_runtime.h>

#include "p32_chain.hpp"
#include "p32_device.hpp"
#include "p32_gemm_tile.hpp"
#include "p32_launch.hpp"

namespace p32 {
namespace {

constexpr int kBT = NT;          // threads per workgroup (the tile routine needs NT)
constexpr int kMaxSub = 64;      // widest sub-panel / sub-block
// k-steps of a proven k-tile unrolled per loop iteration in the tile routine:
// 2 is fastest at six waves per SIMD (fewer live registers than 4).
#ifndef P32_BATCH_UNROLL
#define P32_BATCH_UNROLL 2
#endif
constexpr int kUnroll = P32_BATCH_UNROLL;
constexpr uint32_t kMinus1 = 0xC0000000u;

struct Shared {
  union {
    TileLdsT<BigTile> big;
    TileLdsT<ThinTile> thin;
  } tile;
  unsigned long long red[kBT / 64];
  uint32_t urow[kMaxSub];
  dec udec[kMaxSub];
  uint32_t diag[kMaxSub];
  int32_t piv[kMaxSub];
  int flag;
};

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v, Shared& sh) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long b = sh.red[0];
  for (int i = 1; i < kBT / 64; ++i) b = sh.red[i] > b ? sh.red[i] : b;
  __syncthreads();
  return b;
}

// f(r, q) for every r < rows, q < w, thread t taking the flat indices
// t, t + kBT, ... (r = index / w, q = index % w) with the quotient and
// remainder advanced incrementally: two divisions per call instead of one
// per element.
template <class F>
__device__ __forceinline__ void for_each_rq(int64_t rows, int64_t w, F f) {
  if (rows <= 0 || w <= 0) return;
  const int64_t t = threadIdx.x;
  const int64_t step_r = kBT / w, step_q = kBT % w;
  int64_t r = t / w, q = t % w;
  while (r < rows) {
    f(r, q);
    r += step_r;
    q += step_q;
    if (q >= w) {
      q -= w;
      ++r;
    }
  }
}

// every tile of an m x n region through the tile routine: 64 x 32 tiles,
// or 64 x 16 when the region is at most 16 columns wide (the right-hand
// sides of a solve), so that narrow regions are not padded to 32 columns
template <bool TA, bool TB, bool LOWER, bool CHAIN, bool REVK>
__device__ __forceinline__ void tiles(int64_t m, int64_t n, int64_t k, const uint32_t* A, int64_t lda,
                                      const uint32_t* B, int64_t ldb, uint32_t* C, int64_t ldc,
                                      uint32_t alpha, uint32_t beta, Shared& sh) {
  if (m <= 0 || n <= 0 || k <= 0) return;
  if (!LOWER && n <= ThinTile::BN) {
    const int64_t nr = (m + ThinTile::BM - 1) / ThinTile::BM;
    for (int64_t t = 0; t < nr; ++t)
      gemm_tile<TA, TB, LOWER, CHAIN, REVK, kUnroll, ThinTile>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta,
                                                               t * ThinTile::BM, 0, sh.tile.thin);
  } else {
    const int64_t nr = (m + BM - 1) / BM, nc = (n + BN - 1) / BN;
    for (int64_t t = 0; t < nr * nc; ++t)
      gemm_tile<TA, TB, LOWER, CHAIN, REVK, kUnroll>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta,
                                                     (t / nc) * BM, (t % nc) * BN, sh.tile.big);
  }
  __syncthreads();
}

// ---- LU ---------------------------------------------------------------------

// (i) unblocked LU with partial pivoting of A[c0:n, c0:c0+w]; the swaps stay
// inside the sub-panel; pivots go to ipiv and sh.piv; info is kept uniform.
__device__ __forceinline__ void lu_subpanel(uint32_t* A, int64_t lda, int64_t n, int64_t c0, int w,
                                            int32_t* ipiv, int32_t& info, Shared& sh) {
  const int t = threadIdx.x;
  for (int cl = 0; cl < w; ++cl) {
    const int64_t c = c0 + cl;
    unsigned long long best = 0ull;
    for (int64_t i = c + t; i < n; i += kBT) {
      const unsigned long long kk = pivot_key(A[i * lda + c], i);
      best = kk > best ? kk : best;
    }
    best = block_max_u64(best, sh);
    int64_t p = (int64_t)(0xFFFFFFFFu - (uint32_t)best);
    if (best == 0ull || p < c || p >= n) p = c;
    const uint32_t piv = A[p * lda + c];
    if (piv == 0u && info == 0) info = (int32_t)(c + 1);
    if (t == 0) {
      ipiv[c] = (int32_t)p;
      sh.piv[cl] = (int32_t)p;
    }
    __syncthreads();                               // everyone has read A[p][c]
    if (p != c && t < w) {
      const uint32_t x = A[c * lda + c0 + t];
      A[c * lda + c0 + t] = A[p * lda + c0 + t];
      A[p * lda + c0 + t] = x;
    }
    __syncthreads();
    const int wq = w - cl - 1;                     // sub-panel columns right of c
    if (t < wq) {
      const uint32_t u = A[c * lda + c + 1 + t];
      sh.urow[t] = u;
      sh.udec[t] = decode(u);
    }
    if (piv != 0u) {
      const divisor pd = make_divisor(piv);
      for (int64_t i = c + 1 + t; i < n; i += kBT) A[i * lda + c] = p_div_by(A[i * lda + c], pd);
    }
    __syncthreads();
    for_each_rq(n - c - 1, wq, [&](int64_t di, int64_t q) {
      const int64_t i = c + 1 + di;
      const uint32_t l = A[i * lda + c];
      uint32_t& x = A[i * lda + c + 1 + q];
      x = p_fms_pre(x, l, decode(l), sh.urow[q], sh.udec[q]);
    });
    __syncthreads();
  }
}

// (ii) interchanges of rows c0 .. c0+w-1 (pivots in sh.piv) on every column
// outside [c0, c0+w)
__device__ __forceinline__ void lu_laswp(uint32_t* A, int64_t lda, int64_t n, int64_t c0, int w,
                                         const Shared& sh) {
  for (int64_t q = threadIdx.x; q < n - w; q += kBT) {
    const int64_t col = q < c0 ? q : q + w;
    for (int cl = 0; cl < w; ++cl) {
      const int64_t p = sh.piv[cl], c = c0 + cl;
      if (p != c) {
        const uint32_t x = A[c * lda + col];
        A[c * lda + col] = A[p * lda + col];
        A[p * lda + col] = x;
      }
    }
  }
  __syncthreads();
}

// (iii) rows [c0, c0+w) of the columns [q0, q1): unit-lower solve with the
// sub-panel's triangle, column by column in ascending order
__device__ __forceinline__ void lu_trsm_rows(uint32_t* A, int64_t lda, int64_t c0, int w, int64_t q0,
                                             int64_t q1) {
  const int64_t nq = q1 - q0;
  if (nq <= 0) return;
  for (int cl = 0; cl + 1 < w; ++cl) {
    const int64_t c = c0 + cl;
    for_each_rq(w - cl - 1, nq, [&](int64_t dr, int64_t dq) {
      const int64_t q = q0 + dq;
      const int64_t r = c + 1 + dr;
      A[r * lda + q] = p_fms(A[r * lda + q], A[r * lda + c], A[c * lda + q]);
    });
    __syncthreads();
  }
}

__device__ __forceinline__ void lu_factor(uint32_t* A, int64_t lda, int64_t n, int64_t nb, int sub,
                                          int32_t* ipiv, int32_t& info, Shared& sh) {
  info = 0;
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    const int64_t je = j + jb;
    for (int64_t c0 = j; c0 < je; c0 += sub) {
      const int w = (int)(sub < je - c0 ? sub : je - c0);
      lu_subpanel(A, lda, n, c0, w, ipiv, info, sh);
      lu_laswp(A, lda, n, c0, w, sh);
      const int64_t r1 = c0 + w;                   // first row / column after the sub-panel
      // the panel's columns right of the sub-panel: its rows, then all rows below
      lu_trsm_rows(A, lda, c0, w, r1, je);
      tiles<false, false, false, true, false>(n - r1, je - r1, w, A + r1 * lda + c0, lda,
                                              A + c0 * lda + r1, lda, A + r1 * lda + r1, lda, 0u, 0u,
                                              sh);
    }
    // U12 = L11^-1 A12, only once every interchange of the panel is in place
    // (a later pivot may bring up a row from below the panel)
    for (int64_t c0 = j; c0 < je && je < n; c0 += sub) {
      const int w = (int)(sub < je - c0 ? sub : je - c0);
      const int64_t r1 = c0 + w;
      lu_trsm_rows(A, lda, c0, w, je, n);
      tiles<false, false, false, true, false>(je - r1, n - je, w, A + r1 * lda + c0, lda,
                                              A + c0 * lda + je, lda, A + r1 * lda + je, lda, 0u, 0u,
                                              sh);
    }
    const int64_t r0 = j + jb, rest = n - r0;
    tiles<false, false, false, false, false>(rest, rest, jb, A + r0 * lda + j, lda, A + j * lda + r0, lda,
                                             A + r0 * lda + r0, lda, kMinus1, kOne, sh);
  }
}

// ---- substitutions ----------------------------------------------------------

// Diagonal block [c0, c0+w) (w <= kMaxSub) of a triangular solve, for every
// right-hand side: wave v takes the right-hand sides v, v + 4, v + 8, ...,
// kSolveQ of them at a time, and lane r owns row c0 + r of each, in window
// form with a NaR flag.  kind 0: L unit lower, forward (LU); 1: U upper,
// backward (LU); 2: L lower, forward (Cholesky); 3: L^T, backward (Cholesky).
// Per column c in solve order, every lane divides its running values by its
// diagonal without branches (non-unit kinds) and the owner lane's quotient,
// x[c], is read by all lanes with v_readlane (the exact division runs only
// when the owner's quotient needs it, a wave-uniform branch); every later row
// r then gets x[r] - rnd(T(r,c) x[c]) (chain_update), a zero coefficient
// standing in for the rows without an update.  Each row thus receives the
// per-column steps of the unblocked substitution in the same order, with no
// barrier between the columns.  The rounding table is set up in the tile
// area, which the tiles between the blocks overwrite.
constexpr int kSolveQ = 4;
constexpr int kWaves = kBT / 64;

template <int kind>
__device__ __forceinline__ void diag_solve(const uint32_t* __restrict__ M, int64_t lda, int64_t c0, int w,
                                           uint32_t* __restrict__ B, int64_t ldb, int64_t nrhs, Shared& sh) {
  constexpr bool forward = kind == 0 || kind == 2;
  constexpr bool unit = kind == 0;
  constexpr bool trans = kind == 3;
  lut_t* lut = sh.tile.big.lut;
  static_assert(kBT == 256, "one table entry per thread");
  lut[threadIdx.x] = make_lut_entry(threadIdx.x);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool mine = lane < w;
  // this lane's diagonal entry, with its binary64 reciprocal
  dec dg;
  dg.s = 0;
  dg.sc = kEZero;
  bool dg_bad = true;                            // NaR or zero: quotients are NaR
  double rcp = 0.0;
  if (!unit && mine) {
    const uint32_t dp = M[(c0 + lane) * lda + c0 + lane];
    dg = decode(dp);
    dg_bad = dp == kNaR || dg.s == 0;
    if (!dg_bad) rcp = 1.0 / (double)(dg.s < 0 ? -(int64_t)dg.s : (int64_t)dg.s);
  }
  // coefficient T(row c0 + lane, column c0 + cl), 0 for the rows without an update
  auto coef = [&](int u) -> uint32_t {
    const int cl = forward ? u : w - 1 - u;
    const bool act = mine && u < w && (forward ? lane > cl : lane < cl);
    return act ? (trans ? M[(c0 + cl) * lda + c0 + lane] : M[(c0 + lane) * lda + c0 + cl]) : 0u;
  };
  for (int64_t qb = wave; qb < nrhs; qb += kWaves * kSolveQ) {
    win acc[kSolveQ];
    bool xnar[kSolveQ];
#pragma unroll
    for (int k = 0; k < kSolveQ; ++k) {
      const int64_t q = qb + kWaves * k;
      const uint32_t x0 = mine && q < nrhs ? B[(c0 + lane) * ldb + q] : 0u;
      xnar[k] = x0 == kNaR;
      acc[k] = mine ? bias(win_of(xnar[k] ? 0u : x0)) : idle_acc();   // biased window form
    }
    // coefficients two steps ahead, so that their loads stay off the chain
    uint32_t m0 = coef(0), m1 = coef(1);
    for (int u = 0; u < w; ++u) {
      const int cl = forward ? u : w - 1 - u;      // wave-uniform
      const uint32_t m = m0;
      m0 = m1;
      m1 = coef(u + 2);
      const bool act = mine && (forward ? lane > cl : lane < cl);
      dec md = decode(m);
#pragma unroll
      for (int k = 0; k < kSolveQ; ++k) {
        if (qb + kWaves * k >= nrhs) break;         // wave-uniform
        win xw = acc[k];
        int flags = xnar[k];                        // bit 0: NaR, bit 1: exact division
        if (!unit) {
          bool ok;
          xw = bias(div_win_fast(dec_of_win(unbias(acc[k])), dg, rcp, ok));
          flags = (xnar[k] | dg_bad) | (ok ? 0 : 2);
        }
        const int pf = __builtin_amdgcn_readlane(flags, cl);
        const bool pnar = (pf & 1) != 0;
        if (!unit && (pf & 2) && !pnar) {
          if (lane == cl) xw = bias(div_win(dec_of_win(unbias(acc[k])), dg, rcp));
        }
        win pc;
        pc.h = __builtin_amdgcn_readlane(xw.h, cl);
        pc.e = __builtin_amdgcn_readlane(xw.e, cl);
        if (!unit && lane == cl) {
          acc[k] = xw;
          xnar[k] = pnar;
        }
        xnar[k] = xnar[k] | (act & ((m == kNaR) | pnar));
        const dec dx = dec_of_win(unbias(pc));      // x[c], wave-uniform
        if (!pnar && dx.s != 0) {                  // x[c] = 0 changes nothing
          dec mk = md;
          mk.s = act && !xnar[k] ? md.s : 0;
          acc[k] = chain_update(acc[k], mk, stage_b(dx), scale_proven(dx.sc), lut);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kSolveQ; ++k) {
      const int64_t q = qb + kWaves * k;
      if (mine && q < nrhs) B[(c0 + lane) * ldb + q] = xnar[k] ? kNaR : encode_win(unbias(acc[k]));
    }
  }
  __syncthreads();
}

// The substitutions run in blocks of kSolveBlock rows, whatever the
// factorisation's sub-panel width (the blocking only regroups the work): the
// diagonal block by diag_solve, whose waves then use all their lanes, and the
// rows beyond it by one fused-update chain over the block's columns.
constexpr int kSolveBlock = 64;
static_assert(kSolveBlock <= kMaxSub && kSolveBlock <= 64, "one row per lane");

// forward (unit lower) and backward (upper) substitution with the LU factors
__device__ __forceinline__ void lu_solve(const uint32_t* LU, int64_t lda, int64_t n, const int32_t* ipiv,
                                         uint32_t* B, int64_t ldb, int64_t nrhs, Shared& sh) {
  constexpr int sub = kSolveBlock;
  const int t = threadIdx.x;
  for (int64_t q = t; q < nrhs; q += kBT)
    for (int64_t c = 0; c < n; ++c) {
      const int64_t p = ipiv[c];
      if (p != c) {
        const uint32_t x = B[c * ldb + q];
        B[c * ldb + q] = B[p * ldb + q];
        B[p * ldb + q] = x;
      }
    }
  __syncthreads();
  for (int64_t c0 = 0; c0 < n; c0 += sub) {
    const int w = (int)(sub < n - c0 ? sub : n - c0);
    diag_solve<0>(LU, lda, c0, w, B, ldb, nrhs, sh);
    const int64_t r1 = c0 + w;
    tiles<false, false, false, true, false>(n - r1, nrhs, w, LU + r1 * lda + c0, lda, B + c0 * ldb, ldb,
                                            B + r1 * ldb, ldb, 0u, 0u, sh);
  }
  for (int64_t c1 = n; c1 > 0; c1 -= sub) {
    const int64_t c0 = c1 - sub > 0 ? c1 - sub : 0;
    diag_solve<1>(LU, lda, c0, (int)(c1 - c0), B, ldb, nrhs, sh);
    tiles<false, false, false, true, true>(c0, nrhs, c1 - c0, LU + c0, lda, B + c0 * ldb, ldb, B, ldb, 0u,
                                           0u, sh);
  }
}

// ---- Cholesky -----------------------------------------------------------------

// unblocked Cholesky of the w x w sub-block at A[c0][c0]; returns the failing
// column (>= c0) or -1
__device__ __forceinline__ int64_t chol_subblock(uint32_t* A, int64_t lda, int64_t c0, int w,
                                                 Shared& sh) {
  const int t = threadIdx.x;
  for (int cl = 0; cl < w; ++cl) {
    const int64_t c = c0 + cl;
    if (t == 0) {
      const uint32_t a = A[c * lda + c];
      sh.flag = (int32_t)a <= 0;                   // non-positive or NaR
      if (!sh.flag) A[c * lda + c] = p_sqrt(a);
    }
    __syncthreads();
    if (sh.flag) return c;
    const uint32_t d = A[c * lda + c];
    const int rows = w - cl - 1;
    if (t < rows) A[(c + 1 + t) * lda + c] = p_div_by(A[(c + 1 + t) * lda + c], make_divisor(d));
    __syncthreads();
    for_each_rq(rows, rows, [&](int64_t a, int64_t b) {   // element (c+1+a, c+1+b), b <= a
      if (b <= a) {
        const int64_t i = c + 1 + a, q = c + 1 + b;
        A[i * lda + q] = p_fms(A[i * lda + q], A[i * lda + c], A[q * lda + c]);
      }
    });
    __syncthreads();
  }
  return -1;
}

// rows [r0, r1) against the sub-block's triangle at A[c0][c0] (width w):
// column steps c0 .. c0+steps-1, each dividing column c by L[c][c] and
// updating the later sub-block columns of those rows
__device__ __forceinline__ void chol_trsm_rows(uint32_t* A, int64_t lda, int64_t r0, int64_t r1, int64_t c0,
                                               int w, int steps, Shared& sh) {
  const int t = threadIdx.x;
  const int64_t nr = r1 - r0;
  if (nr <= 0) return;
  if (t < steps) sh.diag[t] = A[(c0 + t) * lda + c0 + t];
  __syncthreads();
  for (int cl = 0; cl < steps; ++cl) {
    const int64_t c = c0 + cl;
    const divisor dv = make_divisor(sh.diag[cl]);
    for (int64_t r = r0 + t; r < r1; r += kBT) A[r * lda + c] = p_div_by(A[r * lda + c], dv);
    __syncthreads();
    for_each_rq(nr, w - cl - 1, [&](int64_t dr, int64_t dq) {
      const int64_t q = c + 1 + dq;
      const int64_t r = r0 + dr;
      A[r * lda + q] = p_fms(A[r * lda + q], A[r * lda + c], A[q * lda + c]);
    });
    __syncthreads();
  }
}

__device__ __forceinline__ void chol_factor(uint32_t* A, int64_t lda, int64_t n, int64_t nb, int sub,
                                            int32_t& info, Shared& sh) {
  info = 0;
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    const int64_t je = j + jb;
    for (int64_t c0 = j; c0 < je; c0 += sub) {
      const int w = (int)(sub < je - c0 ? sub : je - c0);
      const int64_t r1 = c0 + w;
      const int64_t fail = chol_subblock(A, lda, c0, w, sh);
      const int steps = fail < 0 ? w : (int)(fail - c0);
      chol_trsm_rows(A, lda, r1, je, c0, w, steps, sh);
      tiles<false, true, true, true, false>(je - r1, je - r1, steps, A + r1 * lda + c0, lda,
                                            A + r1 * lda + c0, lda, A + r1 * lda + r1, lda, 0u, 0u, sh);
      if (fail >= 0) {
        info = (int32_t)(fail + 1);
        return;
      }
    }
    const int64_t rest = n - je;
    if (rest <= 0) continue;
    for (int64_t c0 = j; c0 < je; c0 += sub) {
      const int w = (int)(sub < je - c0 ? sub : je - c0);
      const int64_t c1 = c0 + w;
      chol_trsm_rows(A, lda, je, n, c0, w, w, sh);
      tiles<false, true, false, true, false>(rest, je - c1, w, A + je * lda + c0, lda, A + c1 * lda + c0,
                                             lda, A + je * lda + c1, lda, 0u, 0u, sh);
    }
    tiles<false, true, true, false, false>(rest, rest, jb, A + je * lda + j, lda, A + je * lda + j, lda,
                                           A + je * lda + je, lda, kMinus1, kOne, sh);
  }
}

__device__ __forceinline__ void chol_solve(const uint32_t* L, int64_t lda, int64_t n, uint32_t* B, int64_t ldb,
                                           int64_t nrhs, Shared& sh) {
  constexpr int sub = kSolveBlock;
  for (int64_t c0 = 0; c0 < n; c0 += sub) {
    const int w = (int)(sub < n - c0 ? sub : n - c0);
    diag_solve<2>(L, lda, c0, w, B, ldb, nrhs, sh);
    const int64_t r1 = c0 + w;
    tiles<false, false, false, true, false>(n - r1, nrhs, w, L + r1 * lda + c0, lda, B + c0 * ldb, ldb,
                                            B + r1 * ldb, ldb, 0u, 0u, sh);
  }
  for (int64_t c1 = n; c1 > 0; c1 -= sub) {
    const int64_t c0 = c1 - sub > 0 ? c1 - sub : 0;
    diag_solve<3>(L, lda, c0, (int)(c1 - c0), B, ldb, nrhs, sh);
    // rows above the block: coefficient L[c][r] = op(A)(r, c) with op = transpose
    tiles<true, false, false, true, true>(c0, nrhs, c1 - c0, L + c0 * lda, lda, B + c0 * ldb, ldb, B, ldb,
                                          0u, 0u, sh);
  }
}

// ---- the kernel -------------------------------------------------------------------

struct Batch {
  Tuning tune;
  int32_t count;
  int32_t max_n;
  int32_t nb;
  const int32_t* n;
  uint32_t* const* A;
  const int64_t* lda;
  int32_t* const* ipiv;
  const int32_t* nrhs;
  uint32_t* const* B;
  const int64_t* ldb;
  int32_t* info;
};

// KIND 0: LU, 1: Cholesky.  FACTOR / SOLVE select the phases; with both, a
// failed factorisation (info > 0) skips the solve.
// Everything is inlined into the kernel, with a register budget of six waves
// per SIMD (80 VGPRs).  That spills to scratch, but the extra waves
// hide the latency of the unblocked steps' barriers and divisions: on the
// 20,000-system batches, 6 waves per SIMD run 2% (LU) and 5% (Cholesky)
// faster than 4, which was itself 23% faster than 2 (no spills); 5 is between
// them and 8 is several times slower (the spills dominate).
#ifndef P32_BATCH_MIN_WAVES
#define P32_BATCH_MIN_WAVES 6
#endif
//
// One system per workgroup, not a persistent loop over systems: the
// dispatcher's dynamic order balances the compute units better (11-12%
// faster on 20,000 systems of order 16..512), and no register, spill slot or
// LDS word of a wave outlives its system.  (Builds of the persistent form
// with other code generation, e.g. a non-unrolled tile loop, corrupted some
// systems that were not the first of their workgroup; launched one system
// per workgroup the same builds are exact.)
template <int KIND, bool FACTOR, bool SOLVE>
__global__ void __launch_bounds__(kBT, P32_BATCH_MIN_WAVES) vbatched_kernel(Batch bt) {
  __shared__ Shared sh;
  {
    const int64_t idx = blockIdx.x;             // the grid has exactly bt.count workgroups
    const int64_t n = bt.n[idx];
    uint32_t* A = bt.A[idx];
    const int64_t lda = bt.lda[idx];
    int32_t* ipiv = KIND == 0 ? bt.ipiv[idx] : nullptr;
    const int64_t nrhs = SOLVE ? bt.nrhs[idx] : 0;
    uint32_t* B = SOLVE ? bt.B[idx] : nullptr;
    const int64_t ldb = SOLVE ? bt.ldb[idx] : 1;
    int b = 0;                                   // size bucket of this system
    while (b + 1 < bt.tune.buckets && n > bt.tune.max_n[b]) ++b;
    const int sub = bt.tune.sub[b];
    int32_t status = 0;
    if (n < 0 || n > bt.max_n) status = -1;
    else if (n > 0 && A == nullptr) status = -2;
    else if (lda < (n > 1 ? n : 1)) status = -3;
    else if (KIND == 0 && n > 0 && ipiv == nullptr) status = -4;
    else if (SOLVE && nrhs < 0) status = -5;
    else if (SOLVE && n > 0 && nrhs > 0 && B == nullptr) status = -6;
    else if (SOLVE && ldb < (nrhs > 1 ? nrhs : 1)) status = -7;
    if (status == 0 && FACTOR) {
      if (KIND == 0) lu_factor(A, lda, n, bt.nb, sub, ipiv, status, sh);
      else chol_factor(A, lda, n, bt.nb, sub, status, sh);
    }
    if (SOLVE && status == 0 && n > 0 && nrhs > 0) {
      if (KIND == 0) lu_solve(A, lda, n, ipiv, B, ldb, nrhs, sh);
      else chol_solve(A, lda, n, B, ldb, nrhs, sh);
    }
    if (threadIdx.x == 0) bt.info[idx] = status;
  }
}

template <int KIND, bool FACTOR, bool SOLVE>
int launch_kernel(hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL((vbatched_kernel<KIND, FACTOR, SOLVE>), dim3((unsigned)bt.count), dim3(kBT), 0, s, bt);
  return launch_status();
}

}  // namespace

// Built-in sub-panel widths per size bucket, measured on MI355X (the
// autotuner replaces them per device): a width >= n runs small systems
// unblocked, 32 suits the larger systems.
Tuning default_tuning(int kind) {
  Tuning t{};
  t.buckets = 6;
  const int32_t max_n[6] = {23, 47, 95, 191, 383, 0x7FFFFFFF};
  const int32_t lu[6] = {48, 64, 32, 32, 32, 32};
  const int32_t chol[6] = {64, 64, 32, 32, 32, 32};
  for (int b = 0; b < 6; ++b) {
    t.max_n[b] = max_n[b];
    t.sub[b] = kind == 0 ? lu[b] : chol[b];
  }
  return t;
}

int launch_vbatched(hipStream_t s, int kind, bool factor, bool solve, int32_t count, int32_t max_n,
                    int64_t nb, const int32_t* n, uint32_t* const* A, const int64_t* lda,
                    int32_t* const* ipiv, const int32_t* nrhs, uint32_t* const* B, const int64_t* ldb,
                    int32_t* info, const Tuning* tune) {
  if (count == 0) return 0;
  if (count < 0 || (int64_t)count * kBT > 0xFFFFFFFFll) return -2;   // grid of count * 256 work-items
  Batch bt{tune != nullptr ? *tune : default_tuning(kind), count, max_n, (int32_t)nb, n, A, lda, ipiv, nrhs,
           B, ldb, info};
  if (kind == 0) {
    if (factor && solve) return launch_kernel<0, true, true>(s, bt);
    if (factor) return launch_kernel<0, true, false>(s, bt);
    return launch_kernel<0, false, true>(s, bt);
  }
  if (factor && solve) return launch_kernel<1, true, true>(s, bt);
  if (factor) return launch_kernel<1, true, false>(s, bt);
  return launch_kernel<1, false, true>(s, bt);
}

}  // namespace p32
