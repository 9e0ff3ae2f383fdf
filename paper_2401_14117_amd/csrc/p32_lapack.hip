// p32_lapack.hip -- blocked Posit(32,2) LU (Rgetrf/Rgetrs) and Cholesky
// (Rpotrf/Rpotrs) on the device, the factorisations whose trailing updates
// the paper accelerates with Rgemm (Section 3, Section 5.2).
//
// The right-looking blocked schedule, with block size nb <= 256, is the one
// stated in the library header; every product and every sum is rounded, and
// every element receives its updates in the stated order, so the results are
// bit-identical to a plain sequential run of that schedule:
//
//  Rgetrf, per panel [j, j+jb): one cooperative launch factors the panel
//    column by column (pivot search over all its rows, swap, scaling, rank-1
//    update of the panel's remaining columns), the rows spread over the
//    workgroups and the pivot candidates exchanged through per-workgroup
//    slots; then the interchanges go to the other columns, U12 = L11^-1 A12
//    (one workgroup per column of A12) and A22 = Rgemm(-1, 1, L21, U12).
//  Rpotrf, per diagonal block, kCholSub columns at a time: the sub-block's
//    unblocked Cholesky in one workgroup, every row below it solved against
//    its triangle (one wave per row), and a fused-update chain over its
//    columns for the rest of the block and the rows below it; then the lower
//    triangle of A22 = Rgemm(-1, 1, L21, L21^T).  A failed diagonal sets
//    info, the block column is restored and refactored unblocked, and every
//    later kernel of the call sees info and does nothing.
//  Rgetrs / Rpotrs: blocked triangular solves -- a diagonal block solved by
//    one workgroup per right-hand side, then the rows outside it updated in
//    parallel, applying the block's columns in the stated order.
// The single fused updates of these unblocked steps take the Rgemm tile's
// k-step arithmetic where it is proven exact (chain_update, p32_chain.hpp).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "p32_chain.hpp"
#include "p32_device.hpp"
#include "p32_gemm_tile.hpp"
#include "p32_launch.hpp"

namespace p32 {

constexpr int kMaxNB = 256;
constexpr uint32_t kMinusOne = 0xC0000000u;

// ---- LU panel --------------------------------------------------------------

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

// v[u] for a wave-uniform u in 0..3, without dynamic register indexing
__device__ __forceinline__ uint32_t pick4(const uint32_t (&v)[4], int u) {
  return u == 0 ? v[0] : u == 1 ? v[1] : u == 2 ? v[2] : v[3];
}
__device__ __forceinline__ void put4(uint32_t (&v)[4], int u, uint32_t x) {
  if (u == 0) v[0] = x;
  else if (u == 1) v[1] = x;
  else if (u == 2) v[2] = x;
  else v[3] = x;
}

#ifndef P32_PANEL_THREADS
#define P32_PANEL_THREADS 512    // threads per panel workgroup
#endif
constexpr int kPanelThreads = P32_PANEL_THREADS;
constexpr int kPanelLds = 16384;        // words of panel rows a workgroup keeps in LDS
constexpr unsigned kPollLimit = 1u << 20;

// Pivot slot of one workgroup for column c: [63:32] the |value| key of its
// best candidate (see pivot_key), [31:8] 0xFFFFFF - row (ties to the smaller
// row), [7:0] c mod 256 as the step tag; 0 in [63:8] means "no candidate".
//
// Everything one workgroup publishes for another (slots and row copies) is
// written and read with agent-scope relaxed atomics, which on gfx950 go to
// the device-coherent level of the memory hierarchy instead of a compute
// unit's or an XCD's private caches.  No ordering between the stores is
// needed: each word of a row copy carries the column it belongs to in its
// high half, so a reader that has seen the slots polls the words it needs
// until they carry the current column.  (Agent-scope fences would order the
// stores but write back and invalidate the whole L2 on every column step,
// ten times the cost; a store-completion wait plus a workgroup barrier
// before the slot store costs one more memory round trip per column.)
__device__ __forceinline__ void publish_tagged(unsigned long long* p, uint32_t c, uint32_t v) {
  __hip_atomic_store(p, ((unsigned long long)c << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the value of a tagged word once it carries column c; late is set when it
// does not within kPollLimit rounds
__device__ __forceinline__ uint32_t await_tagged(const unsigned long long* p, uint32_t c, int& late) {
  unsigned long long v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned rounds = 0; (uint32_t)(v >> 32) != c;) {
    if (++rounds > kPollLimit) {
      late = 1;
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return (uint32_t)v;
}

__device__ __forceinline__ unsigned long long pivot_slot(uint32_t x, int64_t row, int64_t c) {
  const unsigned long long k = pivot_key(x, row) >> 32;
  return (k << 32) | ((unsigned long long)((0xFFFFFFu - (uint32_t)row) & 0xFFFFFFu) << 8) |
         (unsigned long long)(c & 0xFF);
}
__device__ __forceinline__ int64_t slot_row(unsigned long long v) {
  return (int64_t)(0xFFFFFFu - (uint32_t)((v >> 8) & 0xFFFFFFu));
}

// Factorisation of the panel A[j:n, j:j+jb] by one cooperative launch (all
// workgroups resident).  Workgroup w owns the R consecutive rows starting at
// j + w R (in LDS when they fit, else in place in A).  Per column c:
//   1. every workgroup has published its best pivot candidate for column c (a
//      copy of the whole panel row and its slot), and the owner of row c a
//      copy of row c;
//   2. every workgroup waits until all slots carry the tag of column c (this
//      is the only grid-wide synchronisation) and takes the largest;
//   3. the owners of rows c and p swap them from the published copies, and
//      each workgroup scales column c of its rows below c;
//   4. look-ahead: it applies column c's rank-1 update first to column c+1
//      (all its rows below c), picks its candidate for column c+1, completes
//      the update of the two rows it is about to publish (the candidate and
//      row c+1), publishes them (step 1 of column c+1), and only then applies
//      the update to the rest of its rows, while the other workgroups are
//      still publishing.
// Every element still receives column c's update before column c+1's, and
// the pivot search of column c+1 sees column c+1 fully updated, so the order
// of operations is that of the unblocked factorisation.  Other workgroups'
// rows are only read from the published copies; copies and slots are
// double-buffered by the parity of c (a workgroup can be at most one column
// ahead of any other).  A wait that exceeds kPollLimit rounds gives up: info
// is set to -1 and the workgroup exits, so no wave can wait forever.  The
// scaling, the look-ahead update of column c+1 and the candidate search give
// row rr of the workgroup to the same thread, so they need no barrier
// between them.
// Workspace: slot [2][G], crow [2][G][jb], rowc [2][jb], the row copies as
// tagged words, every tag initially 0xFFFFFFFF (no column).
// LDS of the panel factorisation besides the rows themselves
struct PanelShared {
  uint32_t urow[kMaxNB];
  int2 ustg[kMaxNB];                              // urow staged as op(B) operands
  unsigned long long red[2][kPanelThreads / 64];
  lut_t lut[256];
};

// The panel factorisation as run by workgroup w of the G that share the
// panel (tile: the LDS rows when LDS).
template <bool LDS>
__device__ __forceinline__ void lu_panel_body(uint32_t* __restrict__ tile, PanelShared& sh,
                                              uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j,
                                              int jb, int R, const unsigned G, const unsigned w,
                                              unsigned long long* __restrict__ slot,
                                              unsigned long long* __restrict__ crow,
                                              unsigned long long* __restrict__ rowc, int32_t* __restrict__ ipiv,
                                              int32_t* __restrict__ info) {
  auto& urow = sh.urow;
  auto& ustg = sh.ustg;
  auto& red = sh.red;
  auto& lut = sh.lut;

  const int t = threadIdx.x;
  const int64_t r0 = j + (int64_t)w * R;
  const int nr = (int)min((int64_t)R, n - r0);   // >= 1 by the host's choice of G
  uint32_t* T = LDS ? tile : A + r0 * lda + j;
  const int64_t ts = LDS ? jb : lda;              // row stride of T
  int rpar = 0;                                   // parity of the reduction buffer

  if (t < 256) lut[t] = make_lut_entry(t);
  if (LDS) {
    for (int idx = t; idx < nr * jb; idx += kPanelThreads) {
      const int rr = idx / jb, q = idx - rr * jb;
      tile[idx] = A[(r0 + rr) * lda + j + q];
    }
    __syncthreads();
  }

  // largest value over the threads of the workgroup, returned to all of them
  // (one barrier; the buffer alternates so the next call cannot overwrite it
  // while it is still being read)
  auto block_max = [&](unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(v, off);
      v = o > v ? o : v;
    }
    if ((t & 63) == 0) red[rpar][t >> 6] = v;
    __syncthreads();
    unsigned long long b = red[rpar][0];
    for (int i = 1; i < kPanelThreads / 64; ++i) b = red[rpar][i] > b ? red[rpar][i] : b;
    rpar ^= 1;
    return b;
  };

  // this workgroup's candidate for column c (rows >= c, column c up to date;
  // row rs + t + i kPanelThreads goes to thread t, as in the scaling and the
  // look-ahead update)
  auto candidate = [&](int64_t c) {
    const int cl = (int)(c - j);
    unsigned long long best = 0ull;
    for (int rr = (int)max((int64_t)0, c - r0) + t; rr < nr; rr += kPanelThreads) {
      const unsigned long long v = pivot_slot(T[rr * ts + cl], r0 + rr, c);
      best = v > best ? v : best;
    }
    return block_max(best);
  };

  // step 1 for column c: tagged copies of the candidate row and of row c
  // (both up to date in every column), and the slot
  auto publish = [&](int64_t c, unsigned long long best) {
    const int par = (int)(c & 1);
    if ((best >> 8) != 0ull) {
      const int rr = (int)(slot_row(best) - r0);
      unsigned long long* dst = crow + ((size_t)par * G + w) * jb;
      for (int q = t; q < jb; q += kPanelThreads) publish_tagged(dst + q, (uint32_t)c, T[rr * ts + q]);
    }
    if (c >= r0 && c < r0 + nr)
      for (int q = t; q < jb; q += kPanelThreads)
        publish_tagged(rowc + (size_t)par * jb + q, (uint32_t)c, T[(c - r0) * ts + q]);
    if (t == 0) {
      const unsigned long long v = (best >> 8) != 0ull ? best : (unsigned long long)(c & 0xFF);
      __hip_atomic_store(&slot[(size_t)par * G + w], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };

  // step 2 for column c: the winning slot, or 0 after a time-out
  auto await = [&](int64_t c) -> unsigned long long {
    const int par = (int)(c & 1);
    const unsigned long long tag = (unsigned long long)(c & 0xFF);
    unsigned long long mine = 0ull;
    for (unsigned rounds = 0;; ++rounds) {
      int ok = 1;
      mine = 0ull;
      for (unsigned g = t; g < G; g += kPanelThreads) {
        const unsigned long long v =
            __hip_atomic_load(&slot[(size_t)par * G + g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((v & 0xFFull) != tag) ok = 0;
        mine = v > mine ? v : mine;
      }
      if (__syncthreads_and(ok)) break;
      if (rounds >= kPollLimit) return 0ull;
      __builtin_amdgcn_s_sleep(1);
    }
    return block_max(mine);
  };

  // T[rr][q] -= rnd(T[rr][cl] * u_q) (column cl's rank-1 update) for the rows
  // [ra, rb) except skip1 and skip2, and the columns [qa, qb)
  auto update = [&](int cl, int ra, int rb, int qa, int qb, int skip1, int skip2) {
    const int wq = qb - qa;
    const int cnt = rb > ra && wq > 0 ? (rb - ra) * wq : 0;
    for (int idx = t; idx < cnt; idx += kPanelThreads) {
      const int dr = idx / wq;
      const int rr = ra + dr, q = qa + (idx - dr * wq);
      if (rr == skip1 || rr == skip2) continue;
      T[rr * ts + q] = fms_staged(T[rr * ts + q], T[rr * ts + cl], urow[q], ustg[q], lut);
    }
  };

  publish(j, candidate(j));
  for (int cl = 0; cl < jb; ++cl) {
    const int64_t c = j + cl;
    const int par = (int)(c & 1);
    const unsigned long long best = await(c);
    if (best == 0ull) {
      if (t == 0) __hip_atomic_store(info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    int64_t p = slot_row(best);
    if ((best >> 8) == 0ull || p < c || p >= n) p = c;   // (some row >= c always publishes)
    const unsigned wp = (unsigned)((p - j) / R);
    const bool own_c = c >= r0 && c < r0 + nr;
    const bool own_p = p != c && p >= r0 && p < r0 + nr;
    // the pivot row (published copy of row p) becomes row c; row c's copy goes to row p
    int late = 0;
    for (int q = t; q < jb; q += kPanelThreads) {
      const uint32_t u = await_tagged(crow + ((size_t)par * G + wp) * jb + q, (uint32_t)c, late);
      urow[q] = u;
      ustg[q] = stage_b(decode(u));
      if (own_c) T[(c - r0) * ts + q] = u;
      if (own_p) T[(p - r0) * ts + q] = await_tagged(rowc + (size_t)par * jb + q, (uint32_t)c, late);
    }
    if (__syncthreads_or(late)) {
      if (t == 0) __hip_atomic_store(info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const uint32_t piv = urow[cl];
    if (w == 0 && t == 0) {
      ipiv[c] = (int32_t)p;
      if (piv == 0u && *info == 0) *info = (int32_t)(c + 1);
    }
    // rows below c: scale column c
    const int rs = (int)max((int64_t)0, c + 1 - r0);
    if (piv != 0u) {
      const divisor pd = make_divisor(piv);
      for (int rr = rs + t; rr < nr; rr += kPanelThreads) T[rr * ts + cl] = p_div_by(T[rr * ts + cl], pd);
    }
    if (cl + 1 == jb) {
      __syncthreads();                            // before the rows are written back
      break;
    }
    const int64_t c1 = c + 1;
    // look-ahead: column c+1 of every row below c (row rs + idx to thread
    // idx, as in the scaling), then the candidate for it
    update(cl, rs, nr, cl + 1, cl + 2, -1, -1);
    const unsigned long long nbest = candidate(c1);
    // complete the rows about to be published: the candidate and row c+1
    const int rw = (nbest >> 8) != 0ull ? (int)(slot_row(nbest) - r0) : -1;
    const int rc1 = c1 >= r0 && c1 < r0 + nr ? (int)(c1 - r0) : -1;
    {
      const int wq = jb - cl - 2;
      const int rows = (rw >= 0) + (rc1 >= 0 && rc1 != rw);
      for (int idx = t; idx < rows * wq; idx += kPanelThreads) {
        const int k = idx / wq;
        const int rr = (k == 0 && rw >= 0) ? rw : rc1;
        const int q = cl + 2 + (idx - k * wq);
        T[rr * ts + q] = fms_staged(T[rr * ts + q], T[rr * ts + cl], urow[q], ustg[q], lut);
      }
    }
    __syncthreads();
    publish(c1, nbest);
    // the rest of column c's update, while the other workgroups publish
    update(cl, rs, nr, cl + 2, jb, rw, rc1);
    __syncthreads();
  }

  if (LDS)
    for (int idx = t; idx < nr * jb; idx += kPanelThreads) {
      const int rr = idx / jb, q = idx - rr * jb;
      A[(r0 + rr) * lda + j + q] = tile[idx];
    }
}

template <bool LDS>
__global__ void __launch_bounds__(kPanelThreads)
lu_panel_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j, int jb, int R,
                unsigned long long* __restrict__ slot, unsigned long long* __restrict__ crow,
                unsigned long long* __restrict__ rowc, int32_t* __restrict__ ipiv,
                int32_t* __restrict__ info) {
  __shared__ uint32_t tile[LDS ? kPanelLds : 1];
  __shared__ PanelShared sh;
  lu_panel_body<LDS>(tile, sh, A, lda, n, j, jb, R, gridDim.x, blockIdx.x, slot, crow, rowc, ipiv, info);
}

// ---- several systems at once ---------------------------------------------------
// Up to kGroupMax independent LU factorisations advance panel by panel
// together: the panels of all systems at one step in one cooperative launch
// (the workgroups split among the systems, each system with its own exchange
// slots), then one launch each for the interchanges, the U12 solves and the
// trailing updates of every system.  Each system receives exactly the
// operations of its single-matrix factorisation, in the same order.
constexpr int kGroupMax = 16;

struct PanelGroup {
  int count;
  int64_t j;
  int gstart[kGroupMax + 1];                      // first workgroup of each system
  int R[kGroupMax], jb[kGroupMax];
  uint32_t* A[kGroupMax];
  int64_t lda[kGroupMax], n[kGroupMax];
  unsigned long long *slot[kGroupMax], *crow[kGroupMax], *rowc[kGroupMax];
  int32_t *ipiv[kGroupMax], *info[kGroupMax];
};

__device__ __forceinline__ int group_of(const int* start, int count, unsigned b) {
  int s = 0;
  while (s + 1 < count && b >= (unsigned)start[s + 1]) ++s;
  return s;
}

__global__ void __launch_bounds__(kPanelThreads) lu_panel_group_kernel(PanelGroup g) {
  __shared__ uint32_t tile[kPanelLds];
  __shared__ PanelShared sh;
  const int s = group_of(g.gstart, g.count, blockIdx.x);
  const unsigned G = (unsigned)(g.gstart[s + 1] - g.gstart[s]), w = blockIdx.x - (unsigned)g.gstart[s];
  if ((int64_t)g.R[s] * g.jb[s] <= kPanelLds)
    lu_panel_body<true>(tile, sh, g.A[s], g.lda[s], g.n[s], g.j, g.jb[s], g.R[s], G, w, g.slot[s], g.crow[s],
                        g.rowc[s], g.ipiv[s], g.info[s]);
  else
    lu_panel_body<false>(tile, sh, g.A[s], g.lda[s], g.n[s], g.j, g.jb[s], g.R[s], G, w, g.slot[s],
                         g.crow[s], g.rowc[s], g.ipiv[s], g.info[s]);
}

// apply the interchanges of panel [j, j+jb) to the columns outside it
__device__ __forceinline__ void laswp_body(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j,
                                           int64_t jb, const int32_t* __restrict__ ipiv, unsigned bx) {
  int64_t q = (int64_t)bx * blockDim.x + threadIdx.x;
  if (q >= n - jb) return;
  if (q >= j) q += jb;                            // skip the panel's columns
  for (int64_t c = j; c < j + jb; ++c) {
    const int64_t p = ipiv[c];
    if (p != c) {
      const uint32_t x = A[c * lda + q];
      A[c * lda + q] = A[p * lda + q];
      A[p * lda + q] = x;
    }
  }
}

__global__ void laswp_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j, int64_t jb,
                             const int32_t* __restrict__ ipiv) {
  laswp_body(A, lda, n, j, jb, ipiv, blockIdx.x);
}

__global__ void laswp_group_kernel(PanelGroup g) {
  const int s = blockIdx.y;
  laswp_body(g.A[s], g.lda[s], g.n[s], g.j, g.jb[s], g.ipiv[s], blockIdx.x);
}

// U12 = L11^-1 A12 (L11 unit lower, jb x jb at A[j][j]); one workgroup per
// column q of A12, thread r owns row j + r of it and keeps it decoded (window
// form, plus a NaR flag) across the column steps.  Per column c in ascending
// order the owner of row c, final once its own last update is in, publishes
// it through LDS decoded, with its NaR flag (double-buffered by parity); after
// one barrier every row r > c gets x[r] - rnd(L11[r][c] x[c]) (chain_update).
// Each thread reads its own row of L11, contiguous in memory, kTrsmPrefetch
// coefficients ahead.
constexpr int kTrsmPrefetch = 8;

struct TrsmShared {
  int xc_nar[2];
  dec xc_d[2];
  lut_t lut[256];
};

__device__ __forceinline__ void trsm_lu_body(TrsmShared& sh, uint32_t* __restrict__ A, int64_t lda, int64_t j,
                                             int64_t jb, unsigned bx) {
  auto& xc_nar = sh.xc_nar;
  auto& xc_d = sh.xc_d;
  auto& lut = sh.lut;
  const int t = threadIdx.x;
  lut[t] = make_lut_entry(t);
  const int64_t q = j + jb + bx;
  const bool mine = t < jb;
  const uint32_t x0 = mine ? A[(j + t) * lda + q] : 0u;
  bool xnar = x0 == kNaR;
  win acc = mine ? bias(win_of(xnar ? 0u : x0)) : idle_acc();   // biased window form
  const uint32_t* Lrow = A + (j + (mine ? t : 0)) * lda + j;
  uint32_t cur[kTrsmPrefetch], nxt[kTrsmPrefetch];
#pragma unroll
  for (int i = 0; i < kTrsmPrefetch; ++i) cur[i] = i < t && mine ? Lrow[i] : 0u;
  int par = 0;
  for (int c0 = 0; c0 < jb; c0 += kTrsmPrefetch) {
#pragma unroll
    for (int i = 0; i < kTrsmPrefetch; ++i) {
      const int c = c0 + kTrsmPrefetch + i;       // next chunk, only columns left of row t
      nxt[i] = c < t && mine ? Lrow[c] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kTrsmPrefetch; ++i) {
      const int c = c0 + i;
      if (c < jb) {
        if (t == c) {
          xc_nar[par] = xnar;
          xc_d[par] = dec_of_win(unbias(acc));
        }
        __syncthreads();
        if (t > c && mine) {
          const uint32_t l = cur[i];
          const dec dx = xc_d[par];
          if (l == kNaR || xc_nar[par]) xnar = true;
          else if (!xnar && dx.s != 0) acc = chain_update(acc, decode(l), stage_b(dx), scale_proven(dx.sc), lut);
        }
        par ^= 1;
      }
    }
#pragma unroll
    for (int i = 0; i < kTrsmPrefetch; ++i) cur[i] = nxt[i];
  }
  if (mine) A[(j + t) * lda + q] = xnar ? kNaR : encode_win(unbias(acc));
}

__global__ void __launch_bounds__(256)
trsm_lu_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j, int64_t jb) {
  __shared__ TrsmShared sh;
  trsm_lu_body(sh, A, lda, j, jb, blockIdx.x);
}

// column blockIdx.x of system blockIdx.y's A12 (systems with fewer columns
// return at once, the whole workgroup together)
__global__ void __launch_bounds__(256) trsm_lu_group_kernel(PanelGroup g) {
  __shared__ TrsmShared sh;
  const int s = blockIdx.y;
  if ((int64_t)blockIdx.x >= g.n[s] - g.j - g.jb[s]) return;
  trsm_lu_body(sh, g.A[s], g.lda[s], g.j, g.jb[s], blockIdx.x);
}

// ---- Cholesky --------------------------------------------------------------

// Unblocked Cholesky of the diagonal block [j, j+jb) in one workgroup, with
// the block's lower triangle held in LDS (row i at offset i(i+1)/2).  Each
// column step spreads the trailing triangle c < q <= i < jb evenly over the
// threads.  On a non-positive or NaR diagonal the block is written back as it
// stands and info is set.
constexpr int kTri = kMaxNB * (kMaxNB + 1) / 2;
constexpr int kPotf2Threads = 1024;

__device__ __forceinline__ int tri_off(int i) { return i * (i + 1) / 2; }

__global__ void __launch_bounds__(kPotf2Threads)
potf2_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t j, int jb, int32_t* __restrict__ info,
             const uint32_t* __restrict__ saved) {
  __shared__ uint32_t D[kTri];
  __shared__ uint32_t col[kMaxNB];
  __shared__ int2 cstg[kMaxNB];                   // col staged as op(B) operands
  __shared__ lut_t lut[256];
  __shared__ int stop;
  const int t = threadIdx.x;
  if (t < 256) lut[t] = make_lut_entry(t);
  uint32_t* G = A + j * lda + j;
  if (saved == nullptr) {
    if (*info != 0) return;
    for (int i = t >> 6; i < jb; i += kPotf2Threads / 64)
      for (int q = t & 63; q <= i; q += 64) D[tri_off(i) + q] = G[i * lda + q];
  } else {
    // redo the whole block from its saved lower triangle (kept with row
    // stride kMaxNB) when a sub-block of it failed; see launch_potrf
    const int32_t f = *info;
    if (f < j + 1 || f > j + jb) return;
    for (int i = t >> 6; i < jb; i += kPotf2Threads / 64)
      for (int q = t & 63; q <= i; q += 64) D[tri_off(i) + q] = saved[i * kMaxNB + q];
  }
  __syncthreads();
  int c = 0;
  for (; c < jb; ++c) {
    if (t == 0) {
      const uint32_t a = D[tri_off(c) + c];
      stop = (int32_t)a <= 0;                     // non-positive or NaR
      if (stop) *info = (int32_t)(j + c + 1);
      else D[tri_off(c) + c] = p_sqrt(a);
    }
    __syncthreads();
    if (stop) break;
    // the divisor is a positive square root: one binary64 reciprocal serves
    // the whole column's quotients
    const dec dd = decode(D[tri_off(c) + c]);
    const double rcp = 1.0 / (double)dd.s;
    for (int r = c + 1 + t; r < jb; r += kPotf2Threads) {
      const uint32_t a = D[tri_off(r) + c];
      const uint32_t x = a == kNaR ? kNaR : encode_win(div_win(decode(a), dd, rcp));
      D[tri_off(r) + c] = x;
      col[r] = x;
      cstg[r] = stage_b(decode(x));
    }
    __syncthreads();
    // trailing triangle: local row a = i-c-1, local column b = q-c-1 <= a
    const int m = jb - c - 1;
    const int cnt = m * (m + 1) / 2;
    for (int idx = t; idx < cnt; idx += kPotf2Threads) {
      int a = (int)((sqrtf(8.0f * (float)idx + 1.0f) - 1.0f) * 0.5f);
      if (tri_off(a + 1) <= idx) ++a;
      if (tri_off(a) > idx) --a;
      const int i = c + 1 + a, q = c + 1 + (idx - tri_off(a));
      D[tri_off(i) + q] = fms_staged(D[tri_off(i) + q], col[i], col[q], cstg[q], lut);
    }
    __syncthreads();
  }
  for (int i = t >> 6; i < jb; i += kPotf2Threads / 64)
    for (int q = t & 63; q <= i; q += 64) G[i * lda + q] = D[tri_off(i) + q];
}

// L21 = A21 L11^-T for the rows [r_begin, r_end) against the jb x jb triangle
// at A[j][j] (jb <= kCholTrsmMax): one wave per row, lane t holds column
// j + t.  Column by column: x_c = A[r][c] / L[c][c] is final once the updates
// from columns < c are in, then columns c' > c get A[r][c'] - rnd(x_c *
// L[c'][c]) (chain_update).  The triangle is staged in LDS once per
// workgroup (four rows), already decoded; lane c keeps L[c][c] with a binary64
// reciprocal for its quotient, and the new x_c reaches the other lanes through
// v_readlane.
constexpr int kCholTrsmMax = 64;
constexpr int32_t kScNaR = 1 << 20;              // scale field of a staged NaR coefficient

__global__ void __launch_bounds__(256)
trsm_chol_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t r_begin, int64_t r_end, int64_t j,
                 int64_t jb, const int32_t* __restrict__ info) {
  __shared__ int2 Ls[kCholTrsmMax][kCholTrsmMax + 1];   // decoded, NaR as scale kScNaR
  __shared__ lut_t lut[256];
  if (*info != 0) return;
  lut[threadIdx.x] = make_lut_entry((int)threadIdx.x);
  const int lane = threadIdx.x & 63;
  const int w = (int)jb;
  {
    // all of a thread's loads are issued before the first is decoded
    constexpr int kPer = kCholTrsmMax * kCholTrsmMax / 256;
    uint32_t mv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int idx = (int)threadIdx.x + i * 256;
      const int cc = idx / kCholTrsmMax, c = idx % kCholTrsmMax;
      mv[i] = cc < w && c <= cc ? A[(j + cc) * lda + j + c] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int idx = (int)threadIdx.x + i * 256;
      const int cc = idx / kCholTrsmMax, c = idx % kCholTrsmMax;
      if (cc < w && c <= cc) {
        const dec d = decode(mv[i]);
        Ls[cc][c] = make_int2(d.s, mv[i] == kNaR ? kScNaR : d.sc);
      }
    }
  }
  __syncthreads();
  const int64_t r = r_begin + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= r_end) return;
  uint32_t* row = A + r * lda + j;
  // lane c's divisor L[c][c] with its binary64 reciprocal (NaR or zero: NaR quotients)
  dec dg;
  dg.s = 0;
  dg.sc = kEZero;
  bool dg_bad = true;
  double rcp = 0.0;
  if (lane < w) {
    const int2 d2 = Ls[lane][lane];
    dg.s = d2.x;
    dg.sc = d2.y;
    dg_bad = d2.y == kScNaR || d2.x == 0;
    if (!dg_bad) rcp = 1.0 / (double)(dg.s < 0 ? -(int64_t)dg.s : (int64_t)dg.s);
  }
  // lane c's value, kept decoded (biased window form plus a NaR flag)
  const uint32_t v0 = lane < w ? row[lane] : 0u;
  bool vnar = v0 == kNaR;
  win acc = lane < w ? bias(win_of(vnar ? 0u : v0)) : idle_acc();
  int2 mnext = Ls[lane][0];                       // read one step ahead (LDS latency)
  for (int c = 0; c < w; ++c) {
    const int2 m = mnext;
    if (c + 1 < w) mnext = Ls[lane][c + 1];
    if (lane == c) {
      if (dg_bad) vnar = true;
      else if (!vnar) acc = bias(div_win(dec_of_win(unbias(acc)), dg, rcp));
    }
    win xc;
    xc.h = __builtin_amdgcn_readlane(acc.h, c);
    xc.e = __builtin_amdgcn_readlane(acc.e, c);
    const bool xnar = __builtin_amdgcn_readlane((int)vnar, c) != 0;
    const dec dx = dec_of_win(unbias(xc));                 // x_c, wave-uniform
    if (lane > c && lane < w) {
      if (m.y == kScNaR || xnar) vnar = true;
      else if (!vnar && dx.s != 0) {                       // x_c = 0 changes nothing
        dec md;
        md.s = m.x;
        md.sc = m.y;
        acc = chain_update(acc, md, stage_b(dx), scale_proven(dx.sc), lut);
      }
    }
  }
  if (lane < w) row[lane] = vnar ? kNaR : encode_win(unbias(acc));
}

// ---- triangular solves -----------------------------------------------------
// kind 0: L unit lower, forward (getrs);  kind 1: U upper, backward (getrs,
//         and the upper potrs's U)
// kind 2: L lower, forward (potrs);       kind 3: L^T, backward (potrs)
// kind 4: U^T, forward (the transposed getrs, and the upper potrs's U^T)
// kind 5: L^T unit, backward (the transposed getrs)
// T(r, c) is the coefficient of x[c] in row r of the triangular system; the
// transposed kinds (3..5) read it from row c of the stored factor.
__host__ __device__ constexpr bool kind_forward(int kind) { return kind == 0 || kind == 2 || kind == 4; }
__host__ __device__ constexpr bool kind_unit(int kind) { return kind == 0 || kind == 5; }
__host__ __device__ constexpr bool kind_trans(int kind) { return kind >= 3; }

__device__ __forceinline__ uint32_t tri_coef(const uint32_t* M, int64_t lda, int kind, int64_t r,
                                             int64_t c) {
  return kind_trans(kind) ? M[c * lda + r] : M[r * lda + c];
}

// Diagonal block [s, s+bs) (bs <= kTrsvBlock = 64) of the solve for one
// right-hand side q: one wave per right-hand side, lane r owns row s + r and
// keeps it decoded (window form plus a NaR flag).  The block's coefficients
// are staged in LDS once, already decoded, and each lane holds its own
// diagonal entry with a binary64 reciprocal for the quotient estimate.  Per
// column c in solve order, the owner lane of row c (final once its own last
// update is in) divides it by the diagonal (non-unit kinds); the quotient is
// read by every lane with v_readlane (the column index is wave-uniform), and
// every later row r gets x[r] - rnd(T(r,c) x[c]) (chain_update).  No barrier
// on the chain itself.
constexpr int kTrsvBlock = 64;

struct TrsvShared {
  int2 coef[kTrsvBlock][kTrsvBlock + 1];
  lut_t lut[256];
};

template <int kind>
__device__ __forceinline__ void trsv_diag_body(TrsvShared& sh, const uint32_t* __restrict__ M, int64_t lda,
                                               uint32_t* __restrict__ B, int64_t ldb, int64_t s, int bs,
                                               int64_t q) {
  auto& coef = sh.coef;
  auto& lut = sh.lut;
  constexpr bool forward = kind_forward(kind);
  constexpr bool unit = kind_unit(kind);
  const int lane = threadIdx.x;
  // coef[r][u]: coefficient of the u-th column in solve order in row r,
  // decoded; only the entries strictly below the diagonal in solve order are
  // loaded.  The lane index is u (kinds 0..2: a row of M is contiguous) or r
  // (kinds 3..5: a column of M is), and all of a lane's loads are issued
  // before the first is decoded, so the staging waits on memory once, not per
  // row.
  {
    constexpr bool trans = kind_trans(kind);
    uint32_t mv[kTrsvBlock];
#pragma unroll
    for (int a = 0; a < kTrsvBlock; ++a) {
      const int r = trans ? lane : a, u = trans ? a : lane;
      const bool need = a < bs && lane < bs && (forward ? r > u : r + u < bs - 1);
      const int64_t c = forward ? s + u : s + bs - 1 - u;
      mv[a] = need ? tri_coef(M, lda, kind, s + r, c) : 0u;
    }
#pragma unroll
    for (int a = 0; a < kTrsvBlock; ++a) {
      const int r = trans ? lane : a, u = trans ? a : lane;
      if (a < bs && lane < bs) {
        const dec d = decode(mv[a]);
        coef[r][u] = make_int2(d.s, mv[a] == kNaR ? kScNaR : d.sc);
      }
    }
  }
  // this lane's diagonal entry (the divisor when it owns the column)
  dec dg;
  dg.s = 0;
  dg.sc = kEZero;
  bool dg_bad = true;                            // NaR or zero: quotients are NaR
  double rcp = 0.0;
  if (!unit && lane < bs) {
    const uint32_t dp = M[(s + lane) * lda + s + lane];
    dg = decode(dp);
    dg_bad = dp == kNaR || dg.s == 0;
    if (!dg_bad) rcp = 1.0 / (double)(dg.s < 0 ? -(int64_t)dg.s : (int64_t)dg.s);
  }
  const uint32_t x0 = lane < bs ? B[(s + lane) * ldb + q] : 0u;
  bool xnar = x0 == kNaR;
  win acc = lane < bs ? bias(win_of(xnar ? 0u : x0)) : idle_acc();   // biased window form
  for (int i = lane; i < 256; i += kTrsvBlock) lut[i] = make_lut_entry(i);
  __syncthreads();
  // this lane's coefficient of the next step, read one step ahead so that the
  // LDS latency stays off the chain
  int2 mnext = coef[lane][0];
  for (int u = 0; u < bs; ++u) {
    const int cl = forward ? u : bs - 1 - u;                // local column (wave-uniform)
    const int2 m = mnext;
    if (u + 1 < bs) mnext = coef[lane][u + 1];
    // x[c]: the owner's running value, divided by its diagonal (non-unit
    // kinds).  Every lane divides its own running value without branches and
    // the owner's quotient is read with v_readlane, so the chain carries no
    // exec-mask changes; the exact routine runs only when the owner's
    // quotient needs it (a wave-uniform branch).
    win xw = acc;
    int flags = xnar;                                       // bit 0: NaR, bit 1: exact path
    if (!unit) {
      bool ok;
      xw = bias(div_win_fast(dec_of_win(unbias(acc)), dg, rcp, ok));
      flags = (xnar | dg_bad) | (ok ? 0 : 2);
    }
    const int pf = __builtin_amdgcn_readlane(flags, cl);
    const bool pnar = (pf & 1) != 0;
    if (!unit && (pf & 2) && !pnar) {
      if (lane == cl) xw = bias(div_win(dec_of_win(unbias(acc)), dg, rcp));
    }
    win pc;
    pc.h = __builtin_amdgcn_readlane(xw.h, cl);
    pc.e = __builtin_amdgcn_readlane(xw.e, cl);
    if (!unit && lane == cl) {
      acc = xw;
      xnar = pnar;
    }
    // every later row r: x[r] - rnd(T(r,c) x[c]); a zero coefficient (also
    // given to the lanes without an update) leaves the running value as it is
    const bool act = lane < bs && (forward ? lane > cl : lane < cl);
    xnar = xnar | (act & ((m.y == kScNaR) | pnar));
    const dec dx = dec_of_win(unbias(pc));                  // x[c], wave-uniform
    if (!pnar && dx.s != 0) {                              // x[c] = 0 changes nothing
      dec md;
      md.s = act && !xnar ? m.x : 0;
      md.sc = m.y;
      acc = chain_update(acc, md, stage_b(dx), scale_proven(dx.sc), lut);
    }
  }
  if (lane < bs) B[(s + lane) * ldb + q] = xnar ? kNaR : encode_win(unbias(acc));
}

template <int kind>
__global__ void __launch_bounds__(kTrsvBlock)
trsv_diag_kernel(const uint32_t* __restrict__ M, int64_t lda, uint32_t* __restrict__ B, int64_t ldb,
                 int64_t nrhs, int64_t s, int bs) {
  __shared__ TrsvShared sh;
  trsv_diag_body<kind>(sh, M, lda, B, ldb, s, bs, blockIdx.x);
}

// Rows outside the diagonal block [s, s+bs) get that block's columns, in
// ascending order (forward) or descending order (backward).  One wave per 64
// rows and one right-hand side q: lane u holds the block's u-th solved entry
// (in solve order) staged as an op(B) operand, and at step u every lane reads
// it with v_readlane.  Each lane's own coefficients are loaded kTrsvChunk
// steps ahead of its chain of updates, so the chain does not wait on memory
// step by step.  A NaR among the block's entries reaches every row.
constexpr int kTrsvChunk = 16;

// bx: the 64-row chunk of [r0, r1) this workgroup updates; right-hand sides
// q0, q0 + qstep, ... below nrhs
__device__ __forceinline__ void trsv_update_body(lut_t* lut, const uint32_t* __restrict__ M, int64_t lda,
                                                 uint32_t* __restrict__ B, int64_t ldb, int64_t nrhs, int64_t s,
                                                 int bs, int64_t r0, int64_t r1, int kind, unsigned bx,
                                                 int64_t q0, int64_t qstep) {
  for (int i = threadIdx.x; i < 256; i += kTrsvBlock) lut[i] = make_lut_entry(i);
  __syncthreads();
  const bool forward = kind_forward(kind);
  const int lane = threadIdx.x;
  const int64_t r = r0 + (int64_t)bx * kTrsvBlock + lane;
  const bool mine = r < r1;
  const int64_t rr = mine ? r : r0;               // a row in range, for the coefficient loads
  const int64_t cl = forward ? s + lane : s + bs - 1 - lane;
  for (int64_t q = q0; q < nrhs; q += qstep) {
    const uint32_t bl = lane < bs ? B[cl * ldb + q] : 0u;
    const int2 xs = stage_b(decode(bl));          // NaR stages as zero; flagged below
    const bool bnar = __ballot(bl == kNaR) != 0ull;
    const uint32_t x0 = mine ? B[r * ldb + q] : 0u;
    bool xnar = x0 == kNaR || bnar;
    win acc = mine ? bias(win_of(x0 == kNaR ? 0u : x0)) : idle_acc();
    // Coefficient loads are unconditional (steps past the block re-read its
    // last column and are not used), so the compiler sees a straight run of
    // loads and waits only for the chunk it is about to use.
    uint32_t cur[kTrsvChunk], nxt[kTrsvChunk];
#pragma unroll
    for (int i = 0; i < kTrsvChunk; ++i) {
      const int step = min(i, bs - 1);
      cur[i] = tri_coef(M, lda, kind, rr, forward ? s + step : s + bs - 1 - step);
    }
    for (int c0 = 0; c0 < bs; c0 += kTrsvChunk) {
#pragma unroll
      for (int i = 0; i < kTrsvChunk; ++i) {
        const int step = min(c0 + kTrsvChunk + i, bs - 1);
        nxt[i] = tri_coef(M, lda, kind, rr, forward ? s + step : s + bs - 1 - step);
      }
#pragma unroll
      for (int i = 0; i < kTrsvChunk; ++i) {
        const int step = c0 + i;
        if (step < bs) {
          const uint32_t m = cur[i];
          xnar = xnar | (m == kNaR);
          int2 bx;
          bx.x = __builtin_amdgcn_readlane(xs.x, step);
          bx.y = __builtin_amdgcn_readlane(xs.y, step);
          if (bx.x != 0) {                        // wave-uniform; a NaR coefficient updates nothing
            dec md = decode(m);
            md.s = m == kNaR ? 0 : md.s;
            acc = chain_update(acc, md, bx, scale_proven(bx.y >> 4), lut);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < kTrsvChunk; ++i) cur[i] = nxt[i];
    }
    if (mine) B[r * ldb + q] = xnar ? kNaR : encode_win(unbias(acc));
  }
}

__global__ void __launch_bounds__(kTrsvBlock)
trsv_update_kernel(const uint32_t* __restrict__ M, int64_t lda, uint32_t* __restrict__ B, int64_t ldb,
                   int64_t nrhs, int64_t s, int bs, int64_t r0, int64_t r1, int kind) {
  __shared__ lut_t lut[256];
  trsv_update_body(lut, M, lda, B, ldb, nrhs, s, bs, r0, r1, kind, blockIdx.x, blockIdx.y, gridDim.y);
}

// row interchanges of getrs, in order (reverse: in reverse order, which
// undoes them), one thread per right-hand side
__device__ __forceinline__ void apply_pivots_body(uint32_t* __restrict__ B, int64_t ldb, int64_t n,
                                                  int64_t nrhs, const int32_t* __restrict__ ipiv, int reverse,
                                                  int64_t q) {
  if (q >= nrhs) return;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t c = reverse ? n - 1 - t : t;
    const int64_t p = ipiv[c];
    if (p != c) {
      const uint32_t x = B[c * ldb + q];
      B[c * ldb + q] = B[p * ldb + q];
      B[p * ldb + q] = x;
    }
  }
}

__global__ void apply_pivots_kernel(uint32_t* __restrict__ B, int64_t ldb, int64_t n, int64_t nrhs,
                                    const int32_t* __restrict__ ipiv, int reverse) {
  apply_pivots_body(B, ldb, n, nrhs, ipiv, reverse, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// The same interchanges with right-hand side q staged in LDS (n <=
// kPivLdsMax; 8 bytes of LDS per row): the column and the pivot indices are
// loaded by the whole workgroup, one thread makes the swaps in order on LDS
// (a chain of LDS round trips instead of global-memory ones), and the column
// is written back.
constexpr int64_t kPivLdsMax = 8192;

__device__ __forceinline__ void apply_pivots_lds_body(uint32_t* __restrict__ B, int64_t ldb, int64_t n,
                                                      const int32_t* __restrict__ ipiv, int reverse, int64_t q,
                                                      uint32_t* xs, int32_t* ps) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    xs[i] = B[i * ldb + q];
    ps[i] = ipiv[i];
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int64_t t = 0; t < n; ++t) {
      const int64_t c = reverse ? n - 1 - t : t;
      const int64_t p = ps[c];
      if (p != c) {
        const uint32_t x = xs[c];
        xs[c] = xs[p];
        xs[p] = x;
      }
    }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) B[i * ldb + q] = xs[i];
}

__global__ void __launch_bounds__(256)
apply_pivots_lds_kernel(uint32_t* __restrict__ B, int64_t ldb, int64_t n, const int32_t* __restrict__ ipiv,
                        int reverse) {
  extern __shared__ uint32_t piv_lds[];
  apply_pivots_lds_body(B, ldb, n, ipiv, reverse, blockIdx.x, piv_lds, reinterpret_cast<int32_t*>(piv_lds + n));
}

// interchanges of nrhs right-hand sides of an n-row system
static void launch_pivots(hipStream_t s, uint32_t* B, int64_t ldb, int64_t n, int64_t nrhs, const int32_t* ipiv,
                          int reverse) {
  if (n <= kPivLdsMax)
    hipLaunchKernelGGL(apply_pivots_lds_kernel, dim3((unsigned)nrhs), dim3(256), (size_t)n * 8, s, B, ldb, n,
                       ipiv, reverse);
  else
    hipLaunchKernelGGL(apply_pivots_kernel, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, s, B, ldb, n, nrhs,
                       ipiv, reverse);
}

// ---- getrs on several systems at once -------------------------------------------
// The forward and backward substitutions of up to kGroupMax systems advance
// block by block together: at block step b, one launch solves the b-th
// diagonal block (in solve order) of every system that has one, and one
// launch updates every such system's rows beyond it (system = blockIdx.y or
// blockIdx.z).  Each system gets exactly the operations of its own getrs.
struct SolveGroup {
  int count;
  const uint32_t* LU[kGroupMax];
  const int32_t* ipiv[kGroupMax];
  uint32_t* B[kGroupMax];
  int64_t n[kGroupMax], nrhs[kGroupMax], lda[kGroupMax], ldb[kGroupMax];
};

// block b of system s in solve order: its first row and size
__device__ __forceinline__ bool solve_block(const SolveGroup& g, int sys, bool forward, int64_t b, int64_t& s0,
                                            int& bs) {
  const int64_t n = g.n[sys], nblk = (n + kTrsvBlock - 1) / kTrsvBlock;
  if (b >= nblk || g.nrhs[sys] == 0) return false;
  s0 = forward ? b * kTrsvBlock : (nblk - 1 - b) * kTrsvBlock;
  bs = (int)(s0 + kTrsvBlock < n ? kTrsvBlock : n - s0);
  return true;
}

__global__ void apply_pivots_group_kernel(SolveGroup g) {
  const int sys = blockIdx.y;
  apply_pivots_body(g.B[sys], g.ldb[sys], g.n[sys], g.nrhs[sys], g.ipiv[sys], 0,
                    (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// right-hand side blockIdx.x of system blockIdx.y, staged in LDS (every n <= kPivLdsMax)
__global__ void __launch_bounds__(256) apply_pivots_group_lds_kernel(SolveGroup g) {
  extern __shared__ uint32_t piv_lds[];
  const int sys = blockIdx.y;
  const int64_t n = g.n[sys];
  if ((int64_t)blockIdx.x >= g.nrhs[sys]) return;
  apply_pivots_lds_body(g.B[sys], g.ldb[sys], n, g.ipiv[sys], 0, blockIdx.x, piv_lds,
                        reinterpret_cast<int32_t*>(piv_lds + n));
}

template <int kind>
__global__ void __launch_bounds__(kTrsvBlock) trsv_diag_group_kernel(SolveGroup g, int64_t b) {
  __shared__ TrsvShared sh;
  const int sys = blockIdx.y;
  int64_t s0;
  int bs;
  if (!solve_block(g, sys, kind_forward(kind), b, s0, bs) || (int64_t)blockIdx.x >= g.nrhs[sys]) return;
  trsv_diag_body<kind>(sh, g.LU[sys], g.lda[sys], g.B[sys], g.ldb[sys], s0, bs, blockIdx.x);
}

__global__ void __launch_bounds__(kTrsvBlock) trsv_update_group_kernel(SolveGroup g, int64_t b, int kind) {
  __shared__ lut_t lut[256];
  const int sys = blockIdx.z;
  int64_t s0;
  int bs;
  const bool forward = kind_forward(kind);
  if (!solve_block(g, sys, forward, b, s0, bs)) return;
  const int64_t r0 = forward ? s0 + bs : 0, r1 = forward ? g.n[sys] : s0;
  if (r0 + (int64_t)blockIdx.x * kTrsvBlock >= r1) return;
  trsv_update_body(lut, g.LU[sys], g.lda[sys], g.B[sys], g.ldb[sys], g.nrhs[sys], s0, bs, r0, r1, kind,
                   blockIdx.x, blockIdx.y, gridDim.y);
}

__global__ void zero_i32_kernel(int32_t* p) { *p = 0; }

static int trsv(hipStream_t s, const uint32_t* M, int64_t lda, int64_t n, uint32_t* B, int64_t ldb,
                int64_t nrhs, int kind) {
  const int64_t bsz = kTrsvBlock;
  const bool forward = kind_forward(kind);
  const int64_t nblk = (n + bsz - 1) / bsz;
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t s0 = forward ? b * bsz : (nblk - 1 - b) * bsz;
    const int64_t bs = s0 + bsz < n ? bsz : n - s0;
    const dim3 grid((unsigned)nrhs), block(kTrsvBlock);
    if (kind == 0) hipLaunchKernelGGL(trsv_diag_kernel<0>, grid, block, 0, s, M, lda, B, ldb, nrhs, s0, (int)bs);
    else if (kind == 1) hipLaunchKernelGGL(trsv_diag_kernel<1>, grid, block, 0, s, M, lda, B, ldb, nrhs, s0, (int)bs);
    else if (kind == 2) hipLaunchKernelGGL(trsv_diag_kernel<2>, grid, block, 0, s, M, lda, B, ldb, nrhs, s0, (int)bs);
    else if (kind == 3) hipLaunchKernelGGL(trsv_diag_kernel<3>, grid, block, 0, s, M, lda, B, ldb, nrhs, s0, (int)bs);
    else if (kind == 4) hipLaunchKernelGGL(trsv_diag_kernel<4>, grid, block, 0, s, M, lda, B, ldb, nrhs, s0, (int)bs);
    else hipLaunchKernelGGL(trsv_diag_kernel<5>, grid, block, 0, s, M, lda, B, ldb, nrhs, s0, (int)bs);
    const int64_t r0 = forward ? s0 + bs : 0, r1 = forward ? n : s0;
    if (r1 > r0) {
      const unsigned gy = (unsigned)(nrhs < 65535 ? nrhs : 65535);
      hipLaunchKernelGGL(trsv_update_kernel, dim3((unsigned)((r1 - r0 + kTrsvBlock - 1) / kTrsvBlock), gy),
                         dim3(kTrsvBlock), 0, s, M, lda, B, ldb, nrhs, s0, (int)bs, r0, r1, kind);
    }
  }
  return launch_status();
}

// ---- drivers ---------------------------------------------------------------

__global__ void fill_u64_kernel(unsigned long long* p, int64_t count, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

#ifndef P32_PANEL_MIN_ROWS
#define P32_PANEL_MIN_ROWS 4      // fewest panel rows per workgroup
#endif

// The panel's pivot exchange: per workgroup two key slots and two candidate
// rows of 8-byte tagged words, plus two copies of row c -- sized for gmax
// workgroups.
static constexpr size_t getrf_ws_bytes(int64_t gmax) {
  return (size_t)2 * gmax * sizeof(unsigned long long) +
         (size_t)2 * gmax * kMaxNB * sizeof(unsigned long long) +
         (size_t)2 * kMaxNB * sizeof(unsigned long long);
}

// Most workgroups of one panel: one per compute unit (the slot-reading loop
// takes one thread per workgroup), capped at gcap.
static int getrf_setup(int64_t gcap, int* cus, int* per_cu_lds, int* per_cu_glb, int64_t* gmax) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu_lds, reinterpret_cast<const void*>(&lu_panel_kernel<true>), kPanelThreads, 0);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu_glb, reinterpret_cast<const void*>(&lu_panel_kernel<false>), kPanelThreads, 0);
  if (e != hipSuccess) return -1000 - (int)e;
  if (*per_cu_lds < 1 || *per_cu_glb < 1) return -1000 - (int)hipErrorCooperativeLaunchTooLarge;
  int64_t g = *cus < 1 ? 1 : *cus;
  if (g > kPanelThreads) g = kPanelThreads;
  if (g > gcap) g = gcap;
  *gmax = g;
  return 0;
}

// Optional timing of getrf's phases with HIP events recorded between its
// launches: the time from one mark to the next goes to the phase the later
// mark closes (0 panel, 1 interchanges, 2 U12 solve, 3 trailing update).
struct PhaseClock {
  hipStream_t s = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<int> phase;
  int mark(int ph) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    ev.push_back(e);
    phase.push_back(ph);
    return hipEventRecord(e, s) == hipSuccess ? 0 : -1;
  }
  // waits for the last mark; ms[0..3] receive the sums
  int collect(double* ms) {
    for (int i = 0; i < 4; ++i) ms[i] = 0.0;
    int rc = ev.empty() || hipEventSynchronize(ev.back()) == hipSuccess ? 0 : -1;
    for (size_t i = 1; i < ev.size() && rc == 0; ++i) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, ev[i - 1], ev[i]) != hipSuccess) rc = -1;
      else if (phase[i] >= 0 && phase[i] < 4) ms[phase[i]] += t;
    }
    return rc;
  }
  ~PhaseClock() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// getrf on a caller-provided workspace of getrf_ws_bytes(gmax) bytes (every
// word is set before the first panel, so its previous contents do not matter)
static int getrf_run(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                     int32_t* info, char* ws, int64_t gmax, int cus, int per_cu_lds, int per_cu_glb,
                     PhaseClock* clk = nullptr) {
  const size_t slot_bytes = (size_t)2 * gmax * sizeof(unsigned long long);
  const size_t row_bytes = (size_t)2 * gmax * kMaxNB * sizeof(unsigned long long);
  unsigned long long* slot = reinterpret_cast<unsigned long long*>(ws);
  unsigned long long* crow = reinterpret_cast<unsigned long long*>(ws + slot_bytes);
  unsigned long long* rowc = reinterpret_cast<unsigned long long*>(ws + slot_bytes + row_bytes);
  // all ones: slot tag 0xFF matches neither column 0 nor column 1 (every slot
  // is written before the panel's column 255), row-copy tag 0xFFFFFFFF no column
  const int64_t ws_words = (int64_t)(getrf_ws_bytes(gmax) / sizeof(unsigned long long));
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((ws_words + 255) / 256)), dim3(256), 0, s, slot,
                     ws_words, ~0ull);
  int rc = launch_status();
  for (int64_t j = 0; j < n && rc == 0; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    const int64_t rows = n - j;
    int64_t R = (rows + gmax - 1) / gmax;
    if (R < P32_PANEL_MIN_ROWS) R = P32_PANEL_MIN_ROWS;
    const int64_t G = (rows + R - 1) / R;
    const bool lds = R * jb <= kPanelLds;
    if (G > (lds ? per_cu_lds : per_cu_glb) * (int64_t)cus) {
      rc = -1000 - (int)hipErrorCooperativeLaunchTooLarge;
      break;
    }
    int jb_i = (int)jb, R_i = (int)R;
    void* args[] = {&A, &lda, &n, &j, &jb_i, &R_i, &slot, &crow, &rowc, &ipiv, &info};
    const void* fn = lds ? reinterpret_cast<const void*>(&lu_panel_kernel<true>)
                         : reinterpret_cast<const void*>(&lu_panel_kernel<false>);
    if (clk && clk->mark(-1)) rc = -1000 - (int)hipErrorUnknown;
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3((unsigned)G), dim3(kPanelThreads), args, 0, s);
    if (e != hipSuccess) {
      rc = -1000 - (int)e;
      break;
    }
    if (clk && clk->mark(0)) rc = -1000 - (int)hipErrorUnknown;
    if (n - jb > 0)
      hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)((n - jb + 255) / 256)), dim3(256), 0, s, A, lda,
                         n, j, jb, ipiv);
    if (clk && clk->mark(1)) rc = -1000 - (int)hipErrorUnknown;
    const int64_t rest = n - j - jb;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_lu_kernel, dim3((unsigned)rest), dim3(256), 0, s, A, lda, n, j, jb);
      if (clk && clk->mark(2)) rc = -1000 - (int)hipErrorUnknown;
      const int rg = launch_gemm_ex(s, 0, 0, rest, rest, jb, kMinusOne, A + (j + jb) * lda + j, lda,
                                    A + j * lda + j + jb, lda, kOne, A + (j + jb) * lda + j + jb, lda, false,
                                    nullptr);
      if (rc == 0) rc = rg;
      if (clk && clk->mark(3)) rc = -1000 - (int)hipErrorUnknown;
    }
    if (rc == 0) rc = launch_status();
  }
  return rc;
}

int launch_getrf(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                 int32_t* info) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, info);
  if (n == 0) return launch_status();
  int cus = 0, per_cu_lds = 0, per_cu_glb = 0;
  int64_t gmax = 0;
  int rc = getrf_setup(kPanelThreads, &cus, &per_cu_lds, &per_cu_glb, &gmax);
  if (rc != 0) return rc;
  char* ws = nullptr;
  hipError_t e = hipMallocAsync((void**)&ws, getrf_ws_bytes(gmax), s);
  if (e != hipSuccess) return -1000 - (int)e;
  rc = getrf_run(s, n, nb, A, lda, ipiv, info, ws, gmax, cus, per_cu_lds, per_cu_glb);
  e = hipFreeAsync(ws, s);
  if (rc != 0) return rc;
  if (e != hipSuccess) return -1000 - (int)e;
  return launch_status();
}

__global__ void fill_slots_kernel(unsigned long long* p, int count, unsigned long long v) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = v;
}

static_assert(kGetrfGroupMax == kGroupMax, "one system limit for the grouped LU");

// Several LU factorisations advanced panel by panel together.  At panel
// step j every system with n > j takes part: its panel gets a share of the
// panel workgroups proportional to its remaining rows (at least one, at
// least P32_PANEL_MIN_ROWS rows each), and its own exchange slots; the
// interchanges, U12 solves and trailing updates of all systems then go in
// one launch each.  The slots use an 8-bit column tag, and a system's slot
// region moves as the shares change, so every slot is reset before each
// panel step to a tag that neither of the step's first two columns has; the
// row copies carry the full column number, which only grows.
int launch_getrf_group(hipStream_t s, int count, const int64_t* n, int64_t nb, uint32_t* const* A,
                       const int64_t* lda, int32_t* const* ipiv, int32_t* const* info) {
  if (count < 0 || count > kGroupMax) return -1;
  int64_t nmax = 0;
  for (int i = 0; i < count; ++i) {
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, info[i]);
    nmax = n[i] > nmax ? n[i] : nmax;
  }
  if (nmax == 0) return launch_status();
  int cus = 0, per_cu_lds = 0, per_cu_glb = 0, per_cu_group = 0;
  int64_t gmax = 0;
  int rc = getrf_setup(kPanelThreads, &cus, &per_cu_lds, &per_cu_glb, &gmax);
  if (rc != 0) return rc;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu_group, reinterpret_cast<const void*>(&lu_panel_group_kernel), kPanelThreads, 0);
  if (e != hipSuccess) return -1000 - (int)e;
  if (per_cu_group < 1) return -1000 - (int)hipErrorCooperativeLaunchTooLarge;
  if (gmax < count) return -1000 - (int)hipErrorCooperativeLaunchTooLarge;

  const size_t slot_bytes = (size_t)2 * gmax * sizeof(unsigned long long);
  const size_t crow_bytes = (size_t)2 * gmax * kMaxNB * sizeof(unsigned long long);
  const size_t rowc_bytes = (size_t)count * 2 * kMaxNB * sizeof(unsigned long long);
  char* ws = nullptr;
  e = hipMallocAsync((void**)&ws, slot_bytes + crow_bytes + rowc_bytes, s);
  if (e != hipSuccess) return -1000 - (int)e;
  unsigned long long* slot = reinterpret_cast<unsigned long long*>(ws);
  unsigned long long* crow = reinterpret_cast<unsigned long long*>(ws + slot_bytes);
  unsigned long long* rowc = reinterpret_cast<unsigned long long*>(ws + slot_bytes + crow_bytes);
  const int64_t ws_words = (int64_t)((slot_bytes + crow_bytes + rowc_bytes) / sizeof(unsigned long long));
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((ws_words + 255) / 256)), dim3(256), 0, s, slot,
                     ws_words, ~0ull);
  rc = launch_status();
  for (int64_t j = 0; j < nmax && rc == 0; j += nb) {
    PanelGroup g{};
    g.j = j;
    int sys[kGroupMax];
    int64_t rows_total = 0;
    for (int i = 0; i < count; ++i)
      if (n[i] > j) {
        sys[g.count++] = i;
        rows_total += n[i] - j;
      }
    const int64_t budget = gmax - g.count;          // one workgroup each, the rest by rows
    int G = 0;
    int64_t rest_max = 0, cols_max = 0;
    for (int a = 0; a < g.count; ++a) {
      const int i = sys[a];
      const int64_t rows = n[i] - j;
      int64_t Gs = 1 + budget * rows / rows_total;
      int64_t R = (rows + Gs - 1) / Gs;
      if (R < P32_PANEL_MIN_ROWS) R = P32_PANEL_MIN_ROWS;
      Gs = (rows + R - 1) / R;
      g.gstart[a] = G;
      g.R[a] = (int)R;
      g.jb[a] = (int)(nb < rows ? nb : rows);
      g.A[a] = A[i];
      g.lda[a] = lda[i];
      g.n[a] = n[i];
      g.slot[a] = slot + 2 * G;
      g.crow[a] = crow + (size_t)2 * G * kMaxNB;
      g.rowc[a] = rowc + (size_t)i * 2 * kMaxNB;
      g.ipiv[a] = ipiv[i];
      g.info[a] = info[i];
      G += (int)Gs;
      rest_max = rows - g.jb[a] > rest_max ? rows - g.jb[a] : rest_max;
      cols_max = n[i] - g.jb[a] > cols_max ? n[i] - g.jb[a] : cols_max;
    }
    g.gstart[g.count] = G;
    if (G > per_cu_group * (int64_t)cus || G > gmax) {
      rc = -1000 - (int)hipErrorCooperativeLaunchTooLarge;
      break;
    }
    hipLaunchKernelGGL(fill_slots_kernel, dim3(1), dim3(256), 0, s, slot, 2 * G,
                       (unsigned long long)((j + 2) & 0xFF));
    void* args[] = {&g};
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&lu_panel_group_kernel), dim3((unsigned)G),
                                   dim3(kPanelThreads), args, 0, s);
    if (e != hipSuccess) {
      rc = -1000 - (int)e;
      break;
    }
    if (cols_max > 0)
      hipLaunchKernelGGL(laswp_group_kernel, dim3((unsigned)((cols_max + 255) / 256), (unsigned)g.count),
                         dim3(256), 0, s, g);
    if (rest_max > 0) {
      hipLaunchKernelGGL(trsm_lu_group_kernel, dim3((unsigned)rest_max, (unsigned)g.count), dim3(256), 0, s,
                         g);
      int64_t mm[kGroupMax], kk[kGroupMax], ld[kGroupMax];
      const uint32_t* Ap[kGroupMax];
      const uint32_t* Bp[kGroupMax];
      uint32_t* Cp[kGroupMax];
      for (int a = 0; a < g.count; ++a) {
        const int64_t jb = g.jb[a], ldA = g.lda[a];
        mm[a] = g.n[a] - j - jb;
        kk[a] = jb;
        ld[a] = ldA;
        Ap[a] = g.A[a] + (j + jb) * ldA + j;
        Bp[a] = g.A[a] + j * ldA + j + jb;
        Cp[a] = g.A[a] + (j + jb) * ldA + j + jb;
      }
      rc = launch_gemm_group(s, g.count, mm, mm, kk, Ap, ld, Bp, ld, Cp, ld, kMinusOne, kOne);
    }
    if (rc == 0) rc = launch_status();
  }
  e = hipFreeAsync(ws, s);
  if (rc != 0) return rc;
  if (e != hipSuccess) return -1000 - (int)e;
  return launch_status();
}

// getrf with its phases timed (a diagnostic: synchronises the stream)
int launch_getrf_phases(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                        int32_t* info, double* ms) {
  for (int i = 0; i < 4; ++i) ms[i] = 0.0;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, info);
  if (n == 0) return launch_status();
  int cus = 0, per_cu_lds = 0, per_cu_glb = 0;
  int64_t gmax = 0;
  int rc = getrf_setup(kPanelThreads, &cus, &per_cu_lds, &per_cu_glb, &gmax);
  if (rc != 0) return rc;
  char* ws = nullptr;
  hipError_t e = hipMallocAsync((void**)&ws, getrf_ws_bytes(gmax), s);
  if (e != hipSuccess) return -1000 - (int)e;
  PhaseClock clk;
  clk.s = s;
  rc = getrf_run(s, n, nb, A, lda, ipiv, info, ws, gmax, cus, per_cu_lds, per_cu_glb, &clk);
  e = hipFreeAsync(ws, s);
  if (rc == 0 && clk.collect(ms) != 0) rc = -1000 - (int)hipErrorUnknown;
  if (rc != 0) return rc;
  if (e != hipSuccess) return -1000 - (int)e;
  return launch_status();
}

// ---- allocation-free getrf ---------------------------------------------------
// The workspace of getrf in a file-scope device array instead of a
// stream-ordered allocation: sized for kScratchGroups panel workgroups (the
// call caps the panel at that many workgroups, more rows each), 1,056,768
// bytes, held by every GPU the library runs on until the process ends.  In
// host code `scratch` only names the symbol; its device address is taken
// once per device with hipGetSymbolAddress (with that device current) and
// kept in g_scratch, which is what the kernels receive.  Every call on a GPU
// shares that GPU's array.
constexpr int64_t kScratchGroups = 256;
constexpr size_t kScratchBytes = getrf_ws_bytes(kScratchGroups);
static_assert(kScratchBytes == 1056768, "the size the library header states");
static __device__ __align__(256) unsigned long long scratch[kScratchBytes / 8];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices];

static int scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return -1000 - (int)e;
  if (dev < 0 || dev >= kMaxDevices) return -1000 - (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return -1000 - (int)e;
    if (p == nullptr) return -1000 - (int)hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = static_cast<char*>(g_scratch[dev]);
  return 0;
}

int launch_getrf_noalloc(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                         int32_t* info) {
  char* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc != 0) return rc;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, info);
  if (n == 0) return launch_status();
  int cus = 0, per_cu_lds = 0, per_cu_glb = 0;
  int64_t gmax = 0;
  rc = getrf_setup(kScratchGroups, &cus, &per_cu_lds, &per_cu_glb, &gmax);
  if (rc != 0) return rc;
  rc = getrf_run(s, n, nb, A, lda, ipiv, info, ws, gmax, cus, per_cu_lds, per_cu_glb);
  if (rc != 0) return rc;
  return launch_status();
}

// trans == 0: A X = B, i.e. interchanges, L, U.  trans == 1: A^T X = B with
// A^T = U^T L^T P: U^T forward, L^T (unit) backward, then the interchanges
// undone in reverse order.
int launch_getrs(hipStream_t s, int trans, int64_t n, int64_t nrhs, const uint32_t* LU, int64_t lda,
                 const int32_t* ipiv, uint32_t* B, int64_t ldb) {
  if (n == 0 || nrhs == 0) return 0;
  if (trans) {
    int rc = trsv(s, LU, lda, n, B, ldb, nrhs, 4);
    if (rc == 0) rc = trsv(s, LU, lda, n, B, ldb, nrhs, 5);
    if (rc != 0) return rc;
    launch_pivots(s, B, ldb, n, nrhs, ipiv, 1);
    return launch_status();
  }
  launch_pivots(s, B, ldb, n, nrhs, ipiv, 0);
  int rc = trsv(s, LU, lda, n, B, ldb, nrhs, 0);
  if (rc != 0) return rc;
  return trsv(s, LU, lda, n, B, ldb, nrhs, 1);
}

// Rows [j, n) of the block column [j, j+jb) -> dst (row stride kMaxNB):
// inside the diagonal block only its lower triangle, below it whole rows.
// restore: dst -> A for the rows below the block, and only when the block's
// factorisation failed (info in [j+1, j+jb]).
__global__ void save_panel_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t j, int jb, int64_t n,
                                  uint32_t* __restrict__ dst, const int32_t* __restrict__ info,
                                  int restore) {
  const int32_t f = *info;
  if (restore ? (f < j + 1 || f > j + jb) : f != 0) return;
  const int64_t i = blockIdx.x;                  // row j + i
  if (restore && i < jb) return;                 // the block itself is refactored from dst
  const int w = i < jb ? (int)i + 1 : jb;
  for (int q = threadIdx.x; q < w; q += blockDim.x) {
    if (restore) A[(j + i) * lda + j + q] = dst[i * kMaxNB + q];
    else dst[i * kMaxNB + q] = A[(j + i) * lda + j + q];
  }
}

constexpr int64_t kCholSub = 32;     // columns per sub-block of a diagonal block
static_assert(kCholSub <= kCholTrsmMax, "trsm_chol_kernel stages at most kCholTrsmMax columns");

// Rpotrf.  Each diagonal block [j, j+jb) is factored kCholSub columns at a
// time, together with the rows below it: the sub-block's own columns by
// potf2_kernel, every row below the sub-block (the rest of the block and
// L21) by trsm_chol_kernel, and the lower triangle of the rest of the block
// plus the L21 rows by one fused-update chain over the sub-block's columns.
// Every element receives exactly the updates, divisions and square root of
// the unblocked order (the diagonal block unblocked, then L21 row by row), in
// the same sequence.  If a diagonal fails, that order stops inside the
// diagonal block and leaves L21 untouched, so the rows [j, n) of the block
// column are restored from a copy taken before the block started and the
// block is refactored unblocked, which stops at the same column with the
// state the unblocked order leaves.
static int potrf_lower(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info);

// upper == 1: A = U^T U with U in the upper triangle, U = L^T for the lower
// factor L of the symmetric matrix held by A's upper triangle.  The two
// strict triangles are exchanged, the lower form runs (it neither reads nor
// writes the strict upper triangle, which now holds the caller's lower
// triangle), and the triangles are exchanged back: U lands in the upper
// triangle and the strict lower triangle is restored unchanged.
int launch_potrf(hipStream_t s, int upper, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info) {
  if (!upper) return potrf_lower(s, n, nb, A, lda, info);
  int rc = launch_swap_triangles(s, A, lda, n);
  const int rc2 = rc == 0 ? potrf_lower(s, n, nb, A, lda, info) : 0;
  if (rc == 0) rc = launch_swap_triangles(s, A, lda, n);   // also after a failed launch: restore the layout
  return rc2 != 0 ? rc2 : rc;
}

static int potrf_lower(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, info);
  if (n == 0) return launch_status();
  uint32_t* saved = nullptr;
  hipError_t e = hipMallocAsync((void**)&saved, (size_t)n * kMaxNB * sizeof(uint32_t), s);
  if (e != hipSuccess) return -1000 - (int)e;
  int rc = launch_status();
  for (int64_t j = 0; j < n && rc == 0; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    const int64_t je = j + jb;
    hipLaunchKernelGGL(save_panel_kernel, dim3((unsigned)(n - j)), dim3(256), 0, s, A, lda, j, (int)jb, n,
                       saved, info, 0);
    for (int64_t c0 = j; c0 < je && rc == 0; c0 += kCholSub) {
      const int64_t sb = kCholSub < je - c0 ? kCholSub : je - c0;
      hipLaunchKernelGGL(potf2_kernel, dim3(1), dim3(kPotf2Threads), 0, s, A, lda, c0, (int)sb, info,
                         (const uint32_t*)nullptr);
      const int64_t r1 = c0 + sb, below = n - r1;
      if (below > 0) {
        hipLaunchKernelGGL(trsm_chol_kernel, dim3((unsigned)((below + 3) / 4)), dim3(256), 0, s, A, lda,
                           r1, n, c0, sb, info);
        // lower triangle of the rest of the block; every column of it for the
        // rows below the block
        if (je > r1)
          rc = launch_fms_chain(s, 1, below, je - r1, sb, A + r1 * lda + c0, lda, A + r1 * lda + c0, lda,
                                A + r1 * lda + r1, lda, true, info);
      }
    }
    hipLaunchKernelGGL(save_panel_kernel, dim3((unsigned)(n - j)), dim3(256), 0, s, A, lda, j, (int)jb, n,
                       saved, info, 1);
    hipLaunchKernelGGL(potf2_kernel, dim3(1), dim3(kPotf2Threads), 0, s, A, lda, j, (int)jb, info,
                       (const uint32_t*)saved);
    const int64_t rest = n - je;
    if (rest > 0 && rc == 0)
      rc = launch_gemm_ex(s, 0, 1, rest, rest, jb, kMinusOne, A + je * lda + j, lda, A + je * lda + j, lda,
                          kOne, A + je * lda + je, lda, true, info);
    if (rc == 0) rc = launch_status();
  }
  e = hipFreeAsync(saved, s);
  if (rc != 0) return rc;
  if (e != hipSuccess) return -1000 - (int)e;
  return launch_status();
}

int launch_getrs_group(hipStream_t s, int count, const int64_t* n, const int64_t* nrhs, const uint32_t* const* LU,
                       const int64_t* lda, const int32_t* const* ipiv, uint32_t* const* B, const int64_t* ldb) {
  if (count < 0 || count > kGroupMax) return -1;
  SolveGroup g{};
  int64_t nmax = 0, rmax = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] == 0 || nrhs[i] == 0) continue;
    const int c = g.count++;
    g.LU[c] = LU[i];
    g.ipiv[c] = ipiv[i];
    g.B[c] = B[i];
    g.n[c] = n[i];
    g.nrhs[c] = nrhs[i];
    g.lda[c] = lda[i];
    g.ldb[c] = ldb[i];
    nmax = n[i] > nmax ? n[i] : nmax;
    rmax = nrhs[i] > rmax ? nrhs[i] : rmax;
  }
  if (g.count == 0) return 0;
  if (rmax > 65535) return -1;                   // one diagonal workgroup per right-hand side in y
  if (nmax <= kPivLdsMax)
    hipLaunchKernelGGL(apply_pivots_group_lds_kernel, dim3((unsigned)rmax, (unsigned)g.count), dim3(256),
                       (size_t)nmax * 8, s, g);
  else
    hipLaunchKernelGGL(apply_pivots_group_kernel, dim3((unsigned)((rmax + 63) / 64), (unsigned)g.count),
                       dim3(64), 0, s, g);
  const int64_t nblk = (nmax + kTrsvBlock - 1) / kTrsvBlock;
  const unsigned gy = (unsigned)(rmax < 65535 ? rmax : 65535);
  const unsigned gx_upd = (unsigned)((nmax + kTrsvBlock - 1) / kTrsvBlock);
  for (int kind = 0; kind < 2; ++kind)
    for (int64_t b = 0; b < nblk; ++b) {
      if (kind == 0)
        hipLaunchKernelGGL(trsv_diag_group_kernel<0>, dim3((unsigned)rmax, (unsigned)g.count), dim3(kTrsvBlock), 0,
                           s, g, b);
      else
        hipLaunchKernelGGL(trsv_diag_group_kernel<1>, dim3((unsigned)rmax, (unsigned)g.count), dim3(kTrsvBlock), 0,
                           s, g, b);
      hipLaunchKernelGGL(trsv_update_group_kernel, dim3(gx_upd, gy, (unsigned)g.count), dim3(kTrsvBlock), 0, s, g,
                         b, kind);
    }
  return launch_status();
}

// upper == 0: A = L L^T (L forward, L^T backward).  upper == 1: A = U^T U
// with U = L^T: the same two solves reading the factor transposed (U^T
// forward, U backward), so the bits are those of the lower form on the
// transposed factor.
int launch_potrs(hipStream_t s, int upper, int64_t n, int64_t nrhs, const uint32_t* L, int64_t lda,
                 uint32_t* B, int64_t ldb) {
  if (n == 0 || nrhs == 0) return 0;
  int rc = trsv(s, L, lda, n, B, ldb, nrhs, upper ? 4 : 2);
  if (rc != 0) return rc;
  return trsv(s, L, lda, n, B, ldb, nrhs, upper ? 1 : 3);
}

// Exchanges the strict lower and strict upper triangles of the n x n matrix
// A (A[i][j] <-> A[j][i] for i != j), in place.  One workgroup per pair of
// 32 x 32 tiles (bi, bj) with bi >= bj: both tiles are read into LDS with
// coalesced loads and written back transposed into each other's place; a
// diagonal tile is transposed in place.  The diagonal is rewritten with its
// own values.
constexpr int kSwapTile = 32;

__global__ void __launch_bounds__(256)
swap_triangles_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n) {
  __shared__ uint32_t ta[kSwapTile][kSwapTile + 1], tb[kSwapTile][kSwapTile + 1];
  // tile pair t -> (bi, bj) with bi >= bj: t = bi (bi + 1) / 2 + bj
  const int64_t t = blockIdx.x;
  int64_t bi = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) / 2.0);
  while (bi * (bi + 1) / 2 > t) --bi;
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  const int64_t bj = t - bi * (bi + 1) / 2;
  const int64_t i0 = bi * kSwapTile, j0 = bj * kSwapTile;
  const int tx = threadIdx.x % kSwapTile, ty = threadIdx.x / kSwapTile;   // 32 x 8
  for (int r = ty; r < kSwapTile; r += 8) {
    const int64_t gi = i0 + r, gj = j0 + tx;          // tile (bi, bj), row r
    if (gi < n && gj < n) ta[r][tx] = A[gi * lda + gj];
    const int64_t hi = j0 + r, hj = i0 + tx;          // tile (bj, bi), row r
    if (bi != bj && hi < n && hj < n) tb[r][tx] = A[hi * lda + hj];
  }
  __syncthreads();
  for (int r = ty; r < kSwapTile; r += 8) {
    // (bi, bj) receives the transpose of (bj, bi); a diagonal tile its own
    const int64_t gi = i0 + r, gj = j0 + tx;
    if (gi < n && gj < n) A[gi * lda + gj] = bi != bj ? tb[tx][r] : ta[tx][r];
    const int64_t hi = j0 + r, hj = i0 + tx;
    if (bi != bj && hi < n && hj < n) A[hi * lda + hj] = ta[tx][r];
  }
}

int launch_swap_triangles(hipStream_t s, uint32_t* A, int64_t lda, int64_t n) {
  if (n <= 1) return 0;
  const int64_t nt = (n + kSwapTile - 1) / kSwapTile;
  if (nt * (nt + 1) / 2 > 0x7FFFFFFF) return -1000 - (int)hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(swap_triangles_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, A, lda,
                     n);
  return launch_status();
}

}  // namespace p32
