// p32_launch.hpp -- launch helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "posit32.h"

namespace p32 {

// Status of the most recent launch as a library return code.
inline int launch_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -1000 - (int)e;
}

int launch_gemm(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
                const uint32_t* A, int64_t lda, const uint32_t* B, int64_t ldb, uint32_t beta,
                uint32_t* C, int64_t ldc);
int launch_gemm_ex(hipStream_t s, int ta, int tb, int64_t m, int64_t n, int64_t k, uint32_t alpha,
                   const uint32_t* A, int64_t lda, const uint32_t* B, int64_t ldb, uint32_t beta,
                   uint32_t* C, int64_t ldc, bool lower, const int32_t* skip);
// count <= kGemmGroupMax independent problems C_s = alpha A_s B_s + beta C_s
// (no transposes, alpha != 0) in one launch; host arrays, empty problems skipped
constexpr int kGemmGroupMax = 16;
int launch_gemm_group(hipStream_t s, int count, const int64_t* m, const int64_t* n, const int64_t* k,
                      const uint32_t* const* A, const int64_t* lda, const uint32_t* const* B,
                      const int64_t* ldb, uint32_t* const* C, const int64_t* ldc, uint32_t alpha,
                      uint32_t beta);
// C_ij = rnd(C_ij - rnd(A_ip * op(B)_pj)) for p = 0 .. k-1 in order (A not
// transposed; op(B) = B or B^T by tb; lower: only row >= column of C)
int launch_fms_chain(hipStream_t s, int tb, int64_t m, int64_t n, int64_t k, const uint32_t* A,
                     int64_t lda, const uint32_t* B, int64_t ldb, uint32_t* C, int64_t ldc, bool lower,
                     const int32_t* skip);
int launch_from_f64(hipStream_t s, int64_t n, const double* x, uint32_t* out);
int launch_to_f64(hipStream_t s, int64_t n, const uint32_t* p, double* out);
int launch_elementwise(hipStream_t s, int op, int64_t n, const uint32_t* a, const uint32_t* b,
                       uint32_t* out);

int launch_getrf(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                 int32_t* info);
// count <= kGetrfGroupMax independent LU factorisations advanced together
// (host arrays of device pointers); each system's results are those of
// launch_getrf on it
constexpr int kGetrfGroupMax = P32_GROUP_MAX;
int launch_getrf_group(hipStream_t s, int count, const int64_t* n, int64_t nb, uint32_t* const* A,
                       const int64_t* lda, int32_t* const* ipiv, int32_t* const* info);
// getrs (A X = B) on count <= kGetrfGroupMax systems advanced block by block
// together (host arrays); each system's results are those of launch_getrs
int launch_getrs_group(hipStream_t s, int count, const int64_t* n, const int64_t* nrhs, const uint32_t* const* LU,
                       const int64_t* lda, const int32_t* const* ipiv, uint32_t* const* B, const int64_t* ldb);
// getrf with its phases timed by HIP events (ms[4]: panel, interchanges, U12
// solve, trailing update); synchronises the stream
int launch_getrf_phases(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                        int32_t* info, double* ms);
// getrf on the library's file-scope device scratch (no allocation)
int launch_getrf_noalloc(hipStream_t s, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv,
                         int32_t* info);
// trans: solve A^T X = B;  upper: A = U^T U with U in the upper triangle
int launch_getrs(hipStream_t s, int trans, int64_t n, int64_t nrhs, const uint32_t* LU, int64_t lda,
                 const int32_t* ipiv, uint32_t* B, int64_t ldb);
int launch_potrf(hipStream_t s, int upper, int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info);
int launch_potrs(hipStream_t s, int upper, int64_t n, int64_t nrhs, const uint32_t* L, int64_t lda,
                 uint32_t* B, int64_t ldb);
// A[i][j] <-> A[j][i] for every i != j of the n x n matrix A
int launch_swap_triangles(hipStream_t s, uint32_t* A, int64_t lda, int64_t n);

// Sub-panel width per size bucket of the batched kernels: a system of order
// n uses sub[b] for the first bucket b with n <= max_n[b] (else the last).
constexpr int kTuneBuckets = 8;
struct Tuning {
  int32_t buckets;                 // 1 .. kTuneBuckets
  int32_t max_n[kTuneBuckets];     // ascending
  int32_t sub[kTuneBuckets];       // 1 .. 64
};
Tuning default_tuning(int kind);
// validated copy of a table of the C ABI; -1 if it is invalid
int tuning_from_abi(const posit32_vbatch_tuning& t, Tuning* out);

// variable-size batch: kind 0 LU, 1 Cholesky; factor and/or solve phases;
// tune == nullptr takes default_tuning(kind)
int launch_vbatched(hipStream_t s, int kind, bool factor, bool solve, int32_t count, int32_t max_n,
                    int64_t nb, const int32_t* n, uint32_t* const* A, const int64_t* lda,
                    int32_t* const* ipiv, const int32_t* nrhs, uint32_t* const* B, const int64_t* ldb,
                    int32_t* info, const Tuning* tune = nullptr);

}  // namespace p32
