// p32_gemm.hip -- Posit(32,2) Rgemm, C = alpha*op(A)*op(B) + beta*C
// (paper, Section 3, Eq. (2); GPU blocking through shared memory, Section 3.2).
//
// One workgroup of 256 threads owns a BM x BN = 64 x 32 tile of C; each
// thread owns a TM x TN = 4 x 2 micro-tile whose 8 accumulators stay decoded
// in registers (window form) for the whole k loop.  Per k-tile of 16, the
// workgroup reads op(A) and op(B) tiles with coalesced loads, decodes every
// element once into LDS as (significand, scale), and each thread then runs
// the multiply -> round -> add -> round chain for its 8 outputs, strictly in
// ascending k.  NaR inputs
// are recorded per row of op(A) and per column of op(B) (a NaR anywhere in a
// row/column makes the whole output row/column NaR) and replaced by 1.0 in LDS
// so the integer pipeline never sees them.  Rows beyond m and columns beyond
// n are staged as 1.0 (their results are discarded); k beyond the end is
// staged as exact zero, which leaves the accumulators unchanged.
//
// Inside the kernel every window exponent carries the bias EB = 128 (mod 256),
// so that the low byte of an aligned exponent minus the sum's leading-bit
// count indexes the per-workgroup table of rounding parameters (scales
// -124..131), whose entries also hold the biased exponent of the result.  In
// a k-tile whose operands and accumulators are proven to stay in the fast
// range, one k-step per multiply-add is: a 64-bit product, its leading-bit
// count, a table lookup, normalisation with a round-to-odd sticky bit and
// rounding at the table's position; then one shift aligns the smaller of
// product and accumulator, a 32-bit add on the high word forms the exact sum,
// and the same count / lookup / round sequence rounds it.  The k-steps of
// such a tile are unrolled.
#include <hip/hip_runtime.h>

#include "p32_device.hpp"
#include "p32_gemm_tile.hpp"
#include "p32_launch.hpp"

namespace p32 {

// One tile per workgroup.  skip: when non-null and nonzero on entry, the
// kernel does nothing (a failed factorisation step).
// Tiles of a LOWER launch: only the tiles that reach the lower triangle (row
// >= column somewhere in the tile), band by band: band bi (rows 64 bi ..)
// reaches the column tiles 0 .. 2 bi + 1 (BM = 2 BN).  The sequence is cut
// into eight equal chunks, one per XCD as in tile_origin, so every XCD gets
// the same number of tiles; cutting the full rectangle into chunks of bands
// instead would give the bottom band's XCD about fifteen times the work of
// the top one's.
static_assert(BM == 2 * BN, "lower-triangle tile count assumes 64 x 32 tiles");
__host__ __device__ inline int64_t lower_tiles_before(int64_t band, int64_t ncol) {
  const int64_t t = ncol / 2;                    // bands b < t reach 2 b + 2 <= ncol tiles
  return band <= t ? band * (band + 1) : t * (t + 1) + (band - t) * ncol;
}

__device__ __forceinline__ void lower_tile_origin(int64_t m, int64_t n, unsigned g, int64_t& i0,
                                                  int64_t& j0) {
  const int64_t nrow = (m + BM - 1) / BM, ncol = (n + BN - 1) / BN;
  const int64_t G = lower_tiles_before(nrow, ncol);
  if (G % 8 == 0) g = (unsigned)((g % 8u) * (G / 8) + g / 8u);
  int64_t lo = 0, hi = nrow - 1;                 // largest band whose first tile is <= g
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (lower_tiles_before(mid, ncol) <= (int64_t)g) lo = mid;
    else hi = mid - 1;
  }
  i0 = lo * BM;
  j0 = ((int64_t)g - lower_tiles_before(lo, ncol)) * BN;
}

template <bool TA, bool TB, bool LOWER, bool CHAIN>
__global__ void __launch_bounds__(NT, P32_GEMM_MIN_WAVES)
gemm_kernel(int64_t m, int64_t n, int64_t k, const uint32_t* __restrict__ A, int64_t lda,
            const uint32_t* __restrict__ B, int64_t ldb, uint32_t* __restrict__ C, int64_t ldc,
            uint32_t alpha, uint32_t beta, const int32_t* __restrict__ skip) {
  __shared__ TileLds sm;
  if (skip != nullptr && *skip != 0) return;
  int64_t i0, j0;
  if (LOWER) lower_tile_origin(m, n, blockIdx.x, i0, j0);
  else tile_origin(m, n, blockIdx.x, i0, j0);
  gemm_tile<TA, TB, LOWER, CHAIN>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta, i0, j0, sm);
}

// The same tile computation with a smaller workgroup tile (MidTile: 32 x 32
// outputs per 256 threads; SmallTile: 8 x 8 per 64 threads), for shapes whose
// 64 x 32 tiles would leave compute units idle.  Every output still gets the
// one order of operations, so the bits do not depend on the tile shape.
template <bool TA, bool TB, class S>
__global__ void __launch_bounds__(S::NT)
gemm_shape_kernel(int64_t m, int64_t n, int64_t k, const uint32_t* __restrict__ A, int64_t lda,
                  const uint32_t* __restrict__ B, int64_t ldb, uint32_t* __restrict__ C, int64_t ldc,
                  uint32_t alpha, uint32_t beta) {
  __shared__ TileLdsT<S> sm;
  int64_t i0, j0;
  tile_origin<S>(m, n, blockIdx.x, i0, j0);
  gemm_tile<TA, TB, false, false, false, P32_GEMM_UNROLL, S>(m, n, k, A, lda, B, ldb, C, ldc, alpha, beta,
                                                             i0, j0, sm);
}

template <class S>
static int64_t tile_count(int64_t m, int64_t n) {
  return ((m + S::BM - 1) / S::BM) * ((n + S::BN - 1) / S::BN);
}

// Tile shape of a plain Rgemm launch: 64 x 32 tiles while they give every
// compute unit at least four, else 32 x 32 tiles while those give every
// compute unit at least two, else 8 x 8 tiles -- with the latency-bound
// checked k-steps when there are fewer than two of those per compute unit.
// 0 big, 1 mid, 2 small, 3 tiny.
static int pick_shape(int64_t m, int64_t n) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (tile_count<BigTile>(m, n) >= 4 * (int64_t)cus) return 0;
  if (tile_count<MidTile>(m, n) >= 2 * (int64_t)cus) return 1;
  if (tile_count<SmallTile>(m, n) >= 2 * (int64_t)cus) return 2;
  return 3;
}

// Several independent Rgemm problems (no transposes, 64 x 32 tiles) in one
// launch: workgroup b takes tile b - tstart[s] of the problem s whose tile
// range holds b.
struct GemmGroup {
  int count;
  uint32_t alpha, beta;
  unsigned tstart[kGemmGroupMax + 1];
  int64_t m[kGemmGroupMax], n[kGemmGroupMax], k[kGemmGroupMax];
  const uint32_t* A[kGemmGroupMax];
  const uint32_t* B[kGemmGroupMax];
  uint32_t* C[kGemmGroupMax];
  int64_t lda[kGemmGroupMax], ldb[kGemmGroupMax], ldc[kGemmGroupMax];
};

__global__ void __launch_bounds__(NT, P32_GEMM_MIN_WAVES) gemm_group_kernel(GemmGroup g) {
  __shared__ TileLds sm;
  int s = 0;
  while (s + 1 < g.count && blockIdx.x >= g.tstart[s + 1]) ++s;
  int64_t i0, j0;
  tile_origin(g.m[s], g.n[s], blockIdx.x - g.tstart[s], i0, j0);
  gemm_tile<false, false, false, false>(g.m[s], g.n[s], g.k[s], g.A[s], g.lda[s], g.B[s], g.ldb[s], g.C[s],
                                        g.ldc[s], g.alpha, g.beta, i0, j0, sm);
}

int launch_gemm_group(hipStream_t s, int count, const int64_t* m, const int64_t* n, const int64_t* k,
                      const uint32_t* const* A, const int64_t* lda, const uint32_t* const* B,
                      const int64_t* ldb, uint32_t* const* C, const int64_t* ldc, uint32_t alpha,
                      uint32_t beta) {
  if (count < 0 || count > kGemmGroupMax || alpha == 0u) return -1;
  GemmGroup g{};
  g.alpha = alpha;
  g.beta = beta;
  int64_t tiles = 0;
  for (int i = 0; i < count; ++i) {
    if (m[i] <= 0 || n[i] <= 0 || k[i] <= 0) continue;
    const int c = g.count++;
    g.tstart[c] = (unsigned)tiles;
    g.m[c] = m[i];
    g.n[c] = n[i];
    g.k[c] = k[i];
    g.A[c] = A[i];
    g.B[c] = B[i];
    g.C[c] = C[i];
    g.lda[c] = lda[i];
    g.ldb[c] = ldb[i];
    g.ldc[c] = ldc[i];
    tiles += ((m[i] + BM - 1) / BM) * ((n[i] + BN - 1) / BN);
    if (tiles * NT >= ((int64_t)1 << 32)) return -4;
  }
  if (g.count == 0) return 0;
  g.tstart[g.count] = (unsigned)tiles;
  hipLaunchKernelGGL(gemm_group_kernel, dim3((unsigned)tiles), dim3(NT), 0, s, g);
  return launch_status();
}

// alpha == 0 or k == 0: C = (beta == 0) ? 0 : beta*C
__global__ void scale_c_kernel(int64_t m, int64_t n, uint32_t* __restrict__ C, int64_t ldc,
                               uint32_t beta, bool lower, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx / n, j = idx % n;
  if (lower && j > i) return;
  uint32_t& c = C[i * ldc + j];
  if (beta == 0u) { c = 0u; return; }
  if (beta == kNaR || c == kNaR) { c = kNaR; return; }
  c = mul_general(decode(beta), decode(c));
}

int launch_gemm_ex(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
                   const uint32_t* A, int64_t lda, const uint32_t* B, int64_t ldb, uint32_t beta,
                   uint32_t* C, int64_t ldc, bool lower, const int32_t* skip) {
  if (m == 0 || n == 0) return 0;
  if (alpha == 0u || k == 0) {
    const int64_t total = m * n;
    const int threads = 256;
    const int64_t blocks = (total + threads - 1) / threads;
    hipLaunchKernelGGL(scale_c_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, m, n, C, ldc, beta,
                       lower, skip);
    return launch_status();
  }
  const int64_t tiles = lower ? lower_tiles_before((m + BM - 1) / BM, (n + BN - 1) / BN)
                              : ((n + BN - 1) / BN) * ((m + BM - 1) / BM);
  if (tiles * NT >= ((int64_t)1 << 32)) return -4;   // beyond one 1-D launch
  const dim3 grid((unsigned)tiles);
  const dim3 block(NT);
#define P32_LAUNCH(TA_, TB_, LO_) \
  hipLaunchKernelGGL((gemm_kernel<TA_, TB_, LO_, false>), grid, block, 0, s, m, n, k, A, lda, B, ldb, \
                     C, ldc, alpha, beta, skip)
  const int shape = lower ? 0 : pick_shape(m, n);
  if (shape != 0) {
    const int64_t t = shape == 1 ? tile_count<MidTile>(m, n) : tile_count<SmallTile>(m, n);
    const int nt = shape == 1 ? MidTile::NT : SmallTile::NT;
    static_assert(TinyTile::BM == SmallTile::BM && TinyTile::BN == SmallTile::BN, "same tiling");
    if (t * nt >= ((int64_t)1 << 32)) return -4;
#define P32_LAUNCH_S(TA_, TB_, S_) \
    hipLaunchKernelGGL((gemm_shape_kernel<TA_, TB_, S_>), dim3((unsigned)t), dim3(S_::NT), 0, s, m, n, k, A, \
                       lda, B, ldb, C, ldc, alpha, beta)
#define P32_LAUNCH_T(TA_, TB_) \
    if (shape == 1) P32_LAUNCH_S(TA_, TB_, MidTile); \
    else if (shape == 2) P32_LAUNCH_S(TA_, TB_, SmallTile); \
    else P32_LAUNCH_S(TA_, TB_, TinyTile)
    if (!ta && !tb) { P32_LAUNCH_T(false, false); }
    else if (!ta && tb) { P32_LAUNCH_T(false, true); }
    else if (ta && !tb) { P32_LAUNCH_T(true, false); }
    else { P32_LAUNCH_T(true, true); }
#undef P32_LAUNCH_T
#undef P32_LAUNCH_S
    return launch_status();
  }
  if (lower) {
    if (!ta && tb) P32_LAUNCH(false, true, true);
    else return -1;                                   // only the Cholesky form is needed
  } else if (!ta && !tb) P32_LAUNCH(false, false, false);
  else if (!ta && tb) P32_LAUNCH(false, true, false);
  else if (ta && !tb) P32_LAUNCH(true, false, false);
  else P32_LAUNCH(true, true, false);
#undef P32_LAUNCH
  return launch_status();
}

int launch_fms_chain(hipStream_t s, int tb, int64_t m, int64_t n, int64_t k, const uint32_t* A,
                     int64_t lda, const uint32_t* B, int64_t ldb, uint32_t* C, int64_t ldc, bool lower,
                     const int32_t* skip) {
  if (m == 0 || n == 0 || k == 0) return 0;
  const int64_t tiles = lower ? lower_tiles_before((m + BM - 1) / BM, (n + BN - 1) / BN)
                              : ((n + BN - 1) / BN) * ((m + BM - 1) / BM);
  if (tiles * NT >= ((int64_t)1 << 32)) return -4;
  const dim3 grid((unsigned)tiles);
  const dim3 block(NT);
#define P32_LAUNCH(TB_, LO_) \
  hipLaunchKernelGGL((gemm_kernel<false, TB_, LO_, true>), grid, block, 0, s, m, n, k, A, lda, B, ldb, \
                     C, ldc, 0u, 0u, skip)
  if (tb && lower) P32_LAUNCH(true, true);
  else if (tb) P32_LAUNCH(true, false);
  else if (!lower) P32_LAUNCH(false, false);
  else return -1;
#undef P32_LAUNCH
  return launch_status();
}

int launch_gemm(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
                const uint32_t* A, int64_t lda, const uint32_t* B, int64_t ldb, uint32_t beta,
                uint32_t* C, int64_t ldc) {
  return launch_gemm_ex(s, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, false, nullptr);
}

}  // namespace p32
