// p32_gemm.hip -- Posit(32,2) Rgemm, C = alpha*op(A)*op(B) + beta*C
// (paper, Section 3, Eq. (2); GPU blocking through shared memory, Section 3.2).
//
// One workgroup of 256 threads owns a 64 x 64 tile of C; each thread owns a
// 4 x 4 micro-tile whose 16 accumulators stay decoded in registers (window
// form) for the whole k loop.  Per k-tile of 16, the workgroup reads op(A) and
// op(B) tiles with coalesced loads, decodes every element once into LDS as
// (significand, scale), and each thread then runs the multiply -> round ->
// add -> round chain for its 16 outputs, strictly in ascending k.  NaR inputs
// are recorded per row of op(A) and per column of op(B) (a NaR anywhere in a
// row/column makes the whole output row/column NaR) and replaced by 1.0 in LDS
// so the integer pipeline never sees them.  Rows beyond m and columns beyond
// n are staged as 1.0 (their results are discarded); k beyond the end is
// staged as exact zero, which leaves the accumulators unchanged.
#include <hip/hip_runtime.h>

#include "p32_device.hpp"
#include "p32_launch.hpp"

namespace p32 {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256, TM = 4, TN = 4;

// rare path: exact multiply-add for one element
__device__ __noinline__ win madd_slow(win acc, int32_t a8, int32_t sca, int32_t b4, int32_t scb) {
  return add_slow(acc, mul_slow(a8, sca, b4, scb));
}

// epilogue for one element: r = alpha*acc, then r + beta*c
__device__ __noinline__ uint32_t gemm_epilogue(win acc, int nar, uint32_t alpha, uint32_t beta,
                                               uint32_t c) {
  uint32_t r;
  if (nar || alpha == kNaR) {
    r = kNaR;
  } else {
    const uint32_t a = encode_exact(acc);
    r = alpha == kOne ? a : mul_general(decode(alpha), decode(a));
  }
  if (beta != 0u) {
    if (r == kNaR || beta == kNaR || c == kNaR) return kNaR;
    const uint32_t t = mul_general(decode(beta), decode(c));
    r = add_general(win_of(r), win_of(t));
  }
  return r;
}

// One k step for the thread's TM x TN accumulators.  CHECKED also tests the
// product and sum scales and zero products; the unchecked form only tests
// the sum for cancellation (its callers guarantee the rest).  Flagged lanes
// redo the whole step on the exact path.
template <bool CHECKED>
__device__ __forceinline__ void k_step(win (&acc)[TM][TN], const int2* __restrict__ Arow,
                                       const int2* __restrict__ Brow, int tx, int ty) {
  int2 a[TM], b[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) a[i] = Arow[ty * TM + i];
#pragma unroll
  for (int j = 0; j < TN; ++j) b[j] = Brow[tx * TN + j];
  win nacc[TM][TN];
  bool bad = false;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      if (CHECKED) {
        win pr;
        bad |= !mul_fast(a[i].x, a[i].y, b[j].x, b[j].y, pr);
        bad |= !add_fast(acc[i][j], pr, nacc[i][j]);
      } else {
        int c3p, c3;
        const win pr = mul_core(a[i].x, a[i].y, b[j].x, b[j].y, c3p);
        nacc[i][j] = add_core(acc[i][j], pr, c3);
        bad |= (unsigned)c3 >= 29u;
      }
    }
  if (bad) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) nacc[i][j] = madd_slow(acc[i][j], a[i].x, a[i].y, b[j].x, b[j].y);
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = nacc[i][j];
}

template <bool TA, bool TB>
__global__ void __launch_bounds__(NT)
gemm_kernel(int64_t m, int64_t n, int64_t k, const uint32_t* __restrict__ A, int64_t lda,
            const uint32_t* __restrict__ B, int64_t ldb, uint32_t* __restrict__ C, int64_t ldc,
            uint32_t alpha, uint32_t beta) {
  __shared__ int2 As[BK][BM];   // (s << 3, scale) of op(A)(i0 + i, p0 + p)
  __shared__ int2 Bs[BK][BN];   // (s << 2, scale) of op(B)(p0 + p, j0 + j)
  __shared__ int rowNaR[BM], colNaR[BN];

  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int64_t i0 = (int64_t)blockIdx.y * BM, j0 = (int64_t)blockIdx.x * BN;
  if (tid < BM) { rowNaR[tid] = 0; colNaR[tid] = 0; }

  win acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) { acc[i][j].h = 0; acc[i][j].e = kEZero; }

  for (int64_t p0 = 0; p0 < k; p0 += BK) {
    int my_ok = 1;
    __syncthreads();
#pragma unroll
    for (int l = 0; l < (BM * BK) / NT; ++l) {
      const int idx = tid + l * NT;
      const int ii = TA ? idx % BM : idx / BK;
      const int pp = TA ? idx / BM : idx % BK;
      const int64_t gi = i0 + ii, gp = p0 + pp;
      uint32_t v;
      if (gp >= k) v = 0u;
      else if (gi >= m) v = kOne;
      else v = TA ? A[gp * lda + gi] : A[gi * lda + gp];
      if (v == kNaR) { rowNaR[ii] = 1; v = kOne; }
      const dec d = decode(v);
      my_ok &= (d.s != 0) & ((unsigned)(d.sc + 53) <= 102u);
      As[pp][ii] = make_int2(d.s * 8, d.sc);
    }
#pragma unroll
    for (int l = 0; l < (BN * BK) / NT; ++l) {
      const int idx = tid + l * NT;
      const int jj = TB ? idx / BK : idx % BN;
      const int pp = TB ? idx % BK : idx / BN;
      const int64_t gj = j0 + jj, gp = p0 + pp;
      uint32_t v;
      if (gp >= k) v = 0u;
      else if (gj >= n) v = kOne;
      else v = TB ? B[gj * ldb + gp] : B[gp * ldb + gj];
      if (v == kNaR) { colNaR[jj] = 1; v = kOne; }
      const dec d = decode(v);
      my_ok &= (d.s != 0) & ((unsigned)(d.sc + 53) <= 102u);
      Bs[pp][jj] = make_int2(d.s * 4, d.sc);
    }
    // Block-uniform choice of the inner loop for this k-tile.  The unchecked
    // loop is exact when every staged operand is nonzero with scale in
    // [-53, 49] (products then have scales in [-106, 99]) and every
    // accumulator is zero or has scale in [-106, 100].  Sums then keep
    // scales in [-108, 104], inside the fast range: with |p| >= 2^-106, a
    // sum acc + p either has |acc| < |p|/2 and so |sum| > 2^-107, or both
    // terms are multiples of 2^-108 and a nonzero sum is >= 2^-108; and 16
    // products below 2^100 cannot lift |acc| < 2^101 past 2^105.  Only
    // cancellation to zero or by more than 28 bits is left to test.
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        my_ok &= (acc[i][j].h == 0) | ((unsigned)(acc[i][j].e + 106) <= 206u);
    const bool safe = __syncthreads_and(my_ok);

    if (safe) {
#pragma unroll 1
      for (int p = 0; p < BK; ++p) k_step<false>(acc, As[p], Bs[p], tx, ty);
    } else {
#pragma unroll 1
      for (int p = 0; p < BK; ++p) k_step<true>(acc, As[p], Bs[p], tx, ty);
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
      if (gj >= n) continue;
      const int nar = rowNaR[ty * TM + i] | colNaR[tx * TN + j];
      const uint32_t c = beta ? C[gi * ldc + gj] : 0u;
      C[gi * ldc + gj] = gemm_epilogue(acc[i][j], nar, alpha, beta, c);
    }
  }
}

// alpha == 0 or k == 0: C = (beta == 0) ? 0 : beta*C
__global__ void scale_c_kernel(int64_t m, int64_t n, uint32_t* __restrict__ C, int64_t ldc,
                               uint32_t beta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t i = idx / n, j = idx % n;
  uint32_t& c = C[i * ldc + j];
  if (beta == 0u) { c = 0u; return; }
  if (beta == kNaR || c == kNaR) { c = kNaR; return; }
  c = mul_general(decode(beta), decode(c));
}

int launch_gemm(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
                const uint32_t* A, int64_t lda, const uint32_t* B, int64_t ldb, uint32_t beta,
                uint32_t* C, int64_t ldc) {
  if (m == 0 || n == 0) return 0;
  if (alpha == 0u || k == 0) {
    const int64_t total = m * n;
    const int threads = 256;
    const int64_t blocks = (total + threads - 1) / threads;
    hipLaunchKernelGGL(scale_c_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, m, n, C, ldc, beta);
    return launch_status();
  }
  const dim3 grid((unsigned)((n + BN - 1) / BN), (unsigned)((m + BM - 1) / BM));
  const dim3 block(NT);
  if (!ta && !tb) hipLaunchKernelGGL((gemm_kernel<false, false>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, alpha, beta);
  else if (!ta && tb) hipLaunchKernelGGL((gemm_kernel<false, true>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, alpha, beta);
  else if (ta && !tb) hipLaunchKernelGGL((gemm_kernel<true, false>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, alpha, beta);
  else hipLaunchKernelGGL((gemm_kernel<true, true>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, alpha, beta);
  return launch_status();
}

}  // namespace p32
