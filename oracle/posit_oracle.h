/*
 * posit_oracle.h -- reference Posit(N,2) arithmetic and reference BLAS/LAPACK
 * routines.  TEST INFRASTRUCTURE ONLY: the oracle is a plain, slow, obviously
 * correct CPU implementation used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  The GPU library never includes, links or
 * calls anything declared here, and nothing here is derived from the GPU code.
 *
 * Format (paper, Section 2, Eq. (1)): an N-bit posit with es = 2 has the value
 *     x = (-1)^s * u^k * 2^e * 1.f,   u = 2^(2^es) = 16,
 * where the regime is a run of identical bits whose length gives k, followed by
 * a terminating bit, then e_s = 2 exponent bits and f_s fraction bits.  The
 * all-zero pattern is 0 and the pattern 100...0 is NaR ("not a real").
 * Negative values are the two's complement of the pattern of |x|.
 *
 * All patterns are passed as uint32_t holding the N-bit pattern in the low N
 * bits (N = 8, 16 or 32).  Every arithmetic result is the exact result rounded
 * once (round to nearest, ties to the even pattern, never to 0 or NaR).
 */
#ifndef POSIT_ORACLE_H
#define POSIT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- scalar Posit(N,2) operations (N in {8,16,32}) ---------------------- */
uint32_t oracle_posit_add(int N, uint32_t a, uint32_t b);
uint32_t oracle_posit_sub(int N, uint32_t a, uint32_t b);
uint32_t oracle_posit_mul(int N, uint32_t a, uint32_t b);
uint32_t oracle_posit_div(int N, uint32_t a, uint32_t b);
uint32_t oracle_posit_sqrt(int N, uint32_t a);
uint32_t oracle_posit_neg(int N, uint32_t a);
uint32_t oracle_posit_from_double(int N, double x);
double   oracle_posit_to_double(int N, uint32_t a);
/* decoded fields of a pattern: returns 0 normal, 1 zero, 2 NaR */
int      oracle_posit_fields(int N, uint32_t a, int* sign, int* k, int* e,
                             int* fs, uint32_t* f);

/* ---- array helpers (same arithmetic, looped; OpenMP over elements) ----- */
void oracle_vec_from_double(int N, int64_t n, const double* x, uint32_t* out);
void oracle_vec_to_double(int N, int64_t n, const uint32_t* p, double* out);
/* op: 0 add, 1 sub, 2 mul, 3 div, 4 sqrt (b ignored) */
void oracle_vec_binop(int N, int op, int64_t n, const uint32_t* a,
                      const uint32_t* b, uint32_t* out);

/* ---- Rgemm: C = alpha*op(A)*op(B) + beta*C (paper, Section 3, Eq. (2)) --
 * Posit(32,2), row-major storage, op(X) = X (0) or X^T (1).
 * Per element: acc = 0; for p = 0..k-1 ascending: acc = add(acc, mul(a, b));
 * r = mul(alpha, acc); C = (beta == 0) ? r : add(r, mul(beta, C)).
 * alpha == 0 or k == 0: C = (beta == 0) ? 0 : mul(beta, C); A, B not read.
 * beta == 0: C is not read.  Rows are distributed over OpenMP threads; the
 * order of operations inside one element never changes.                     */
void oracle_gemm(int transa, int transb, int64_t m, int64_t n, int64_t k,
                 uint32_t alpha, const uint32_t* A, int64_t lda,
                 const uint32_t* B, int64_t ldb, uint32_t beta,
                 uint32_t* C, int64_t ldc);
/* Same arithmetic for a list of (row, col) entries only.  Cin holds the input
 * C values of those entries, out receives the results.                       */
void oracle_gemm_entries(int transa, int transb, int64_t k, uint32_t alpha,
                         const uint32_t* A, int64_t lda, const uint32_t* B,
                         int64_t ldb, uint32_t beta, int64_t count,
                         const int64_t* rows, const int64_t* cols,
                         const uint32_t* Cin, uint32_t* out);

/* ---- factorisations and solves (Posit(32,2), row-major) ----------------
 * Right-looking blocked algorithms with block size nb; ref_lapack.c states
 * the order of every operation.  ipiv is 0-based: row c was interchanged
 * with row ipiv[c].  info: 0 ok; >0 = 1-based column of the first zero pivot
 * (getrf, which completes) or of the first non-positive/NaR diagonal
 * (potrf, which stops there).  potrf/potrs use the lower triangle only.  */
void oracle_getrf(int64_t n, int64_t nb, uint32_t* A, int64_t lda,
                  int32_t* ipiv, int32_t* info);
void oracle_getrs(int64_t n, int64_t nrhs, const uint32_t* LU, int64_t lda,
                  const int32_t* ipiv, uint32_t* B, int64_t ldb);
void oracle_potrf(int64_t n, int64_t nb, uint32_t* A, int64_t lda,
                  int32_t* info);
void oracle_potrs(int64_t n, int64_t nrhs, const uint32_t* L, int64_t lda,
                  uint32_t* B, int64_t ldb);
/* the transposed solve and the upper Cholesky forms (order in ref_lapack.c) */
void oracle_getrs_trans(int64_t n, int64_t nrhs, const uint32_t* LU, int64_t lda,
                        const int32_t* ipiv, uint32_t* B, int64_t ldb);
int oracle_potrf_upper(int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info);
void oracle_potrs_upper(int64_t n, int64_t nrhs, const uint32_t* U, int64_t lda, uint32_t* B,
                        int64_t ldb);

/* number of OpenMP threads the oracle's parallel loops use */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
