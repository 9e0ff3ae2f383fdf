// p32_lapack.hip -- blocked Posit(32,2) LU (Rgetrf/Rgetrs) and Cholesky
// (Rpotrf/Rpotrs) on the device, the factorisations whose trailing updates
// the paper accelerates with Rgemm (Section 3, Section 5.2).
//
// The right-looking blocked schedule, with block size nb <= 256, is the one
// stated in the library header; every product and every sum is rounded, and
// every element receives its updates in the stated order, so the results are
// bit-identical to a plain sequential run of that schedule:
//
//  Rgetrf, per panel [j, j+jb):
//    for each column c: pivot search (argmax |A[i][c]| in posit order over
//    i >= c, ties to the smallest row; a 64-bit atomic max per wave), row
//    swap inside the panel, scaling of the column by the pivot, rank-1
//    update of the panel's remaining columns -- fused with the pivot search
//    of the next column;
//    interchanges applied to the other columns; U12 = L11^-1 A12 (one wave
//    per column of A12); trailing update A22 = Rgemm(-1, 1, L21, U12).
//  Rpotrf, per diagonal block: unblocked Cholesky of the block in one
//    workgroup; L21 = A21 L11^-T (one wave per row of A21); lower triangle of
//    A22 = Rgemm(-1, 1, L21, L21^T).  A failed diagonal sets info and every
//    later kernel of the call sees it and does nothing.
//  Rgetrs / Rpotrs: blocked triangular solves -- a diagonal block solved by
//    one workgroup, then the rows outside it updated in parallel, applying
//    the block's columns in the stated order.
#include <hip/hip_runtime.h>

#include "p32_device.hpp"
#include "p32_launch.hpp"

namespace p32 {

constexpr int kMaxNB = 256;
constexpr uint32_t kMinusOne = 0xC0000000u;

// ---- LU panel --------------------------------------------------------------

__device__ inline void wave_atomic_max(unsigned long long* dst, unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  if ((threadIdx.x & 63) == 0 && v != 0ull) atomicMax(dst, v);
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

// pivot key of column c over rows [c, n)
__global__ void argmax_kernel(const uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t c,
                              unsigned long long* __restrict__ key) {
  unsigned long long best = 0ull;
  for (int64_t i = c + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long kk = pivot_key(A[i * lda + c], i);
    best = kk > best ? kk : best;
  }
  wave_atomic_max(key, best);
}

// record the pivot of column c and swap rows c and p inside the panel
__global__ void panel_swap_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t c,
                                  int64_t j, int64_t jb, const unsigned long long* __restrict__ key,
                                  int32_t* __restrict__ ipiv, int32_t* __restrict__ info) {
  const unsigned long long kc = key[c];
  int64_t p = (int64_t)(0xFFFFFFFFu - (uint32_t)(kc & 0xFFFFFFFFull));
  if (kc == 0ull || p < c || p >= n) p = c;       // (a search always sets the key)
  const uint32_t abs_pivot = (uint32_t)(kc >> 32) ^ 0x80000000u;   // |pivot| pattern
  const int t = threadIdx.x;
  if (t == 0) {
    ipiv[c] = (int32_t)p;
    if (abs_pivot == 0u && *info == 0) *info = (int32_t)(c + 1);
  }
  if (p != c && t < jb) {
    const int64_t q = j + t;
    const uint32_t x = A[c * lda + q];
    A[c * lda + q] = A[p * lda + q];
    A[p * lda + q] = x;
  }
}

// rows (c, n): scale column c by the pivot, rank-1 update of the panel
// columns (c, j+jb), and the pivot key of column c+1
__global__ void __launch_bounds__(256)
panel_update_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t c, int64_t j,
                    int64_t jb, unsigned long long* __restrict__ key) {
  __shared__ uint32_t urow[kMaxNB];
  const int64_t qend = j + jb;
  const int64_t w = qend - c - 1;                 // columns to update
  for (int64_t t = threadIdx.x; t < w; t += blockDim.x) urow[t] = A[c * lda + c + 1 + t];
  __syncthreads();
  const uint32_t piv = A[c * lda + c];
  unsigned long long best = 0ull;
  const int64_t i = c + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    uint32_t* row = A + i * lda;
    uint32_t l = row[c];
    if (piv != 0u) {
      l = p_div(l, piv);
      row[c] = l;
    }
    for (int64_t t = 0; t < w; ++t) row[c + 1 + t] = p_fms(row[c + 1 + t], l, urow[t]);
    if (w > 0) best = pivot_key(row[c + 1], i);
  }
  if (w > 0) wave_atomic_max(key + c + 1, best);
}

// apply the interchanges of panel [j, j+jb) to the columns outside it
__global__ void laswp_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j, int64_t jb,
                             const int32_t* __restrict__ ipiv) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// U12 = L11^-1 A12 (L11 unit lower, jb x jb at A[j][j]); one wave per column
// of A12; lane t holds rows j + t + 64 u of the column
__global__ void __launch_bounds__(256)
trsm_lu_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j, int64_t jb) {
  const int lane = threadIdx.x & 63;
  const int64_t q = j + jb + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= n) return;
  uint32_t v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = lane + 64 * u;
    v[u] = r < jb ? A[(j + r) * lda + q] : 0u;
  }
  for (int c = 0; c < jb; ++c) {
    const uint32_t bc = __shfl(pick4(v, c >> 6), c & 63);   // final value of row c
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = lane + 64 * u;
      if (r > c && r < jb) v[u] = p_fms(v[u], A[(j + r) * lda + j + c], bc);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = lane + 64 * u;
    if (r < jb) A[(j + r) * lda + q] = v[u];
  }
}

// ---- Cholesky --------------------------------------------------------------

// unblocked Cholesky of the diagonal block [j, j+jb) in one workgroup
__global__ void __launch_bounds__(1024)
potf2_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t j, int64_t jb, int32_t* __restrict__ info) {
  __shared__ uint32_t dsh;
  __shared__ int stop;
  if (*info != 0) return;
  const int t = threadIdx.x;
  uint32_t* D = A + j * lda + j;
  for (int c = 0; c < jb; ++c) {
    if (t == 0) {
      const uint32_t a = D[c * lda + c];
      stop = (int32_t)a <= 0;                     // non-positive or NaR
      if (stop) {
        *info = (int32_t)(j + c + 1);
      } else {
        dsh = p_sqrt(a);
        D[c * lda + c] = dsh;
      }
    }
    __syncthreads();
    if (stop) return;
    const uint32_t d = dsh;
    for (int i = c + 1 + t; i < jb; i += blockDim.x) D[i * lda + c] = p_div(D[i * lda + c], d);
    __syncthreads();
    // lower triangle c < q <= i < jb: 32 row lanes x 32 column lanes
    const int ri = t >> 5, qi = t & 31;
    for (int i = c + 1 + ri; i < jb; i += 32)
      for (int q = c + 1 + qi; q <= i; q += 32)
        D[i * lda + q] = p_fms(D[i * lda + q], D[i * lda + c], D[q * lda + c]);
    __syncthreads();
  }
}

// L21 = A21 L11^-T: one wave per row of A21; lane t holds columns t + 64 u.
// Column by column: x_c = A[r][c] / L[c][c] is final once the updates from
// columns < c are in, then columns c' > c get A[r][c'] - rnd(x_c * L[c'][c]).
__global__ void __launch_bounds__(256)
trsm_chol_kernel(uint32_t* __restrict__ A, int64_t lda, int64_t n, int64_t j, int64_t jb,
                 const int32_t* __restrict__ info) {
  if (*info != 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t r = j + jb + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  uint32_t* row = A + r * lda + j;
  const uint32_t* L = A + j * lda + j;
  uint32_t v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = lane + 64 * u;
    v[u] = c < jb ? row[c] : 0u;
  }
  for (int c = 0; c < jb; ++c) {
    uint32_t xc = 0u;
    if ((c & 63) == lane) {
      xc = p_div(pick4(v, c >> 6), L[c * lda + c]);
      put4(v, c >> 6, xc);
    }
    xc = __shfl(xc, c & 63);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cc = lane + 64 * u;
      if (cc > c && cc < jb) v[u] = p_fms(v[u], xc, L[cc * lda + c]);
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = lane + 64 * u;
    if (c < jb) row[c] = v[u];
  }
}

// ---- triangular solves -----------------------------------------------------
// kind 0: L unit lower, forward (getrs);  kind 1: U upper, backward (getrs)
// kind 2: L lower, forward (potrs);       kind 3: L^T, backward (potrs)
// T(r, c) is the coefficient of x[c] in row r of the triangular system.

__device__ __forceinline__ uint32_t tri_coef(const uint32_t* M, int64_t lda, int kind, int64_t r,
                                             int64_t c) {
  return kind == 3 ? M[c * lda + r] : M[r * lda + c];
}

// diagonal block [s, s+bs) of the solve, all right-hand sides, one workgroup
__global__ void __launch_bounds__(256)
trsv_diag_kernel(const uint32_t* __restrict__ M, int64_t lda, uint32_t* __restrict__ B, int64_t ldb,
                 int64_t nrhs, int64_t s, int64_t bs, int kind) {
  const bool forward = kind == 0 || kind == 2;
  const bool unit = kind == 0;
  const int t = threadIdx.x;
  for (int64_t step = 0; step < bs; ++step) {
    const int64_t c = forward ? s + step : s + bs - 1 - step;
    if (!unit)
      for (int64_t q = t; q < nrhs; q += blockDim.x)
        B[c * ldb + q] = p_div(B[c * ldb + q], M[c * lda + c]);
    __syncthreads();
    const int64_t r0 = forward ? c + 1 : s, r1 = forward ? s + bs : c;
    const int64_t cnt = (r1 - r0) * nrhs;
    for (int64_t idx = t; idx < cnt; idx += blockDim.x) {
      const int64_t r = r0 + idx / nrhs, q = idx % nrhs;
      B[r * ldb + q] = p_fms(B[r * ldb + q], tri_coef(M, lda, kind, r, c), B[c * ldb + q]);
    }
    __syncthreads();
  }
}

// rows outside the diagonal block [s, s+bs) get that block's columns, in
// ascending order (forward) or descending order (backward)
__global__ void trsv_update_kernel(const uint32_t* __restrict__ M, int64_t lda, uint32_t* __restrict__ B,
                                   int64_t ldb, int64_t nrhs, int64_t s, int64_t bs, int64_t r0,
                                   int64_t r1, int kind) {
  const bool forward = kind == 0 || kind == 2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (r1 - r0) * nrhs) return;
  const int64_t r = r0 + idx / nrhs, q = idx % nrhs;
  uint32_t x = B[r * ldb + q];
  for (int64_t step = 0; step < bs; ++step) {
    const int64_t c = forward ? s + step : s + bs - 1 - step;
    x = p_fms(x, tri_coef(M, lda, kind, r, c), B[c * ldb + q]);
  }
  B[r * ldb + q] = x;
}

// row interchanges of getrs, in order, one thread per right-hand side
__global__ void apply_pivots_kernel(uint32_t* __restrict__ B, int64_t ldb, int64_t n, int64_t nrhs,
                                    const int32_t* __restrict__ ipiv) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nrhs) return;
  for (int64_t c = 0; c < n; ++c) {
    const int64_t p = ipiv[c];
    if (p != c) {
      const uint32_t x = B[c * ldb + q];
      B[c * ldb + q] = B[p * ldb + q];
      B[p * ldb + q] = x;
    }
  }
}

__global__ void zero_i32_kernel(int32_t* p) { *p = 0; }

static int trsv(hipStream_t s, const uint32_t* M, int64_t lda, int64_t n, uint32_t* B, int64_t ldb,
                int64_t nrhs, int kind) {
  const int64_t bsz = 256;
  const bool forward = kind == 0 || kind == 2;
  const int64_t nblk = (n + bsz - 1) / bsz;
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t s0 = forward ? b * bsz : (nblk - 1 - b) * bsz;
    const int64_t bs = s0 + bsz < n ? bsz : n - s0;
    hipLaunchKernelGGL(trsv_diag_kernel, dim3(1), dim3(256), 0, s, M, lda, B, ldb, nrhs, s0, bs, kind);
    const int64_t r0 = forward ? s0 + bs : 0, r1 = forward ? n : s0;
    const int64_t cnt = (r1 - r0) * nrhs;
    if (cnt > 0)
      hipLaunchKernelGGL(trsv_update_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, M,
                         lda, B, ldb, nrhs, s0, bs, r0, r1, kind);
  }
  return launch_status();
}

// ---- drivers ---------------------------------------------------------------

int launch_getrf(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                 int32_t* info) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, info);
  if (n == 0) return launch_status();
  unsigned long long* keys = nullptr;
  hipError_t e = hipMallocAsync((void**)&keys, (size_t)n * sizeof(unsigned long long), s);
  if (e != hipSuccess) return -1000 - (int)e;
  e = hipMemsetAsync(keys, 0, (size_t)n * sizeof(unsigned long long), s);
  if (e != hipSuccess) return -1000 - (int)e;
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    const unsigned g0 = (unsigned)((n - j + 255) / 256);
    hipLaunchKernelGGL(argmax_kernel, dim3(g0 < 64 ? g0 : 64), dim3(256), 0, s, A, lda, n, j, keys + j);
    for (int64_t c = j; c < j + jb; ++c) {
      hipLaunchKernelGGL(panel_swap_kernel, dim3(1), dim3(256), 0, s, A, lda, n, c, j, jb, keys, ipiv,
                         info);
      const int64_t rows = n - c - 1;
      if (rows > 0)
        hipLaunchKernelGGL(panel_update_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s,
                           A, lda, n, c, j, jb, keys);
    }
    if (n - jb > 0)
      hipLaunchKernelGGL(laswp_kernel, dim3((unsigned)((n - jb + 255) / 256)), dim3(256), 0, s, A, lda,
                         n, j, jb, ipiv);
    const int64_t rest = n - j - jb;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_lu_kernel, dim3((unsigned)((rest + 3) / 4)), dim3(256), 0, s, A, lda, n, j,
                         jb);
      const int rc = launch_gemm_ex(s, 0, 0, rest, rest, jb, kMinusOne, A + (j + jb) * lda + j, lda,
                                    A + j * lda + j + jb, lda, kOne, A + (j + jb) * lda + j + jb, lda,
                                    false, nullptr);
      if (rc != 0) return rc;
    }
    const int rc = launch_status();
    if (rc != 0) return rc;
  }
  e = hipFreeAsync(keys, s);
  if (e != hipSuccess) return -1000 - (int)e;
  return launch_status();
}

int launch_getrs(hipStream_t s, int64_t n, int64_t nrhs, const uint32_t* LU, int64_t lda,
                 const int32_t* ipiv, uint32_t* B, int64_t ldb) {
  if (n == 0 || nrhs == 0) return 0;
  hipLaunchKernelGGL(apply_pivots_kernel, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, s, B, ldb, n,
                     nrhs, ipiv);
  int rc = trsv(s, LU, lda, n, B, ldb, nrhs, 0);
  if (rc != 0) return rc;
  return trsv(s, LU, lda, n, B, ldb, nrhs, 1);
}

int launch_potrf(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, s, info);
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    hipLaunchKernelGGL(potf2_kernel, dim3(1), dim3(1024), 0, s, A, lda, j, jb, info);
    const int64_t rest = n - j - jb;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_chol_kernel, dim3((unsigned)((rest + 3) / 4)), dim3(256), 0, s, A, lda, n,
                         j, jb, info);
      const int rc = launch_gemm_ex(s, 0, 1, rest, rest, jb, kMinusOne, A + (j + jb) * lda + j, lda,
                                    A + (j + jb) * lda + j, lda, kOne, A + (j + jb) * lda + j + jb, lda,
                                    true, info);
      if (rc != 0) return rc;
    }
    const int rc = launch_status();
    if (rc != 0) return rc;
  }
  return launch_status();
}

int launch_potrs(hipStream_t s, int64_t n, int64_t nrhs, const uint32_t* L, int64_t lda, uint32_t* B,
                 int64_t ldb) {
  if (n == 0 || nrhs == 0) return 0;
  int rc = trsv(s, L, lda, n, B, ldb, nrhs, 2);
  if (rc != 0) return rc;
  return trsv(s, L, lda, n, B, ldb, nrhs, 3);
}

}  // namespace p32
