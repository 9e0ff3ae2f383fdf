/*
 * posit32.h -- C ABI of libposit32.so, Posit(32,2) dense linear algebra on
 * AMD Instinct MI355X (gfx950).
 *
 * Number format: Posit(32,2) (paper, Section 2, Eq. (1)):
 *   x = (-1)^s * 16^k * 2^e * 1.f,
 * a 32-bit pattern holding the sign, a regime run of m identical bits closed by
 * the opposite bit (k = m-1 for ones, k = -m for zeros), two exponent bits and
 * 28 - m fraction bits.  0x00000000 is zero, 0x80000000 is NaR, 0x40000000 is
 * 1.0, 0x7FFFFFFF is maxpos = 2^120, 0x00000001 is minpos = 2^-120, and a
 * negative value is the two's complement of the pattern of its magnitude.
 * Every operation returns the exact result rounded once to the nearest posit,
 * ties to the even pattern, never to 0 or NaR (|x| >= maxpos gives maxpos,
 * 0 < |x| <= minpos gives minpos).  NaR in any operand gives NaR.
 *
 * Conventions for every entry point:
 *   - Matrices are raw posit patterns (uint32_t), ROW-MAJOR, with a leading
 *     dimension (row stride, in elements) >= the row width.
 *   - All matrix and vector pointers are DEVICE pointers owned by the caller
 *     (e.g. torch int32 tensors); the library never frees or retains them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls enqueue work on that stream and return without synchronising;
 *     a return of 0 means "enqueued".
 *   - Arguments are validated on the host before anything is launched.  A
 *     negative return -i means "argument i (1-based, counting stream as 1)
 *     is invalid" and nothing was launched.  P32_E_HIP - e (e > 0, a
 *     hipError_t) reports a HIP runtime failure at launch.
 *   - Calls that overlap on one stream are ordered; the library keeps no
 *     global mutable state, so calls on different streams may run
 *     concurrently on disjoint outputs.
 */
#ifndef POSIT32_H
#define POSIT32_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef uint32_t posit32_t;

enum { P32_NOTRANS = 0, P32_TRANS = 1 };
enum { P32_LOWER = 0, P32_UPPER = 1 };

#define P32_OK 0
#define P32_E_HIP (-1000)           /* P32_E_HIP - hipError_t */

/* Library version as 10000*major + 100*minor + patch. */
int posit32_version(void);

/* Human-readable text for a return code (static storage). */
const char* posit32_strerror(int code);

/*
 * posit32_gemm -- C = alpha * op(A) * op(B) + beta * C   (paper, Section 3,
 * Eq. (2), the Level-3 BLAS GEMM interface; the four transpose combinations
 * of Section 3.2).
 *
 *   transa, transb  P32_NOTRANS: op(X) = X;  P32_TRANS: op(X) = X^T.
 *   m, n, k         op(A) is m x k, op(B) is k x n, C is m x n; each >= 0.
 *   A, lda          op(A) = A: A is m x k with lda >= max(1, k);
 *                   op(A) = A^T: A is k x m with lda >= max(1, m).
 *   B, ldb          op(B) = B: B is k x n with ldb >= max(1, n);
 *                   op(B) = B^T: B is n x k with ldb >= max(1, k).
 *   C, ldc          m x n, ldc >= max(1, n); read (unless beta == 0) and
 *                   written.  C must not alias A or B.
 *
 * Order of operations (the result is unique and bit-reproducible):
 *   for each (i, j):  acc = 0;
 *                     for p = 0, 1, ..., k-1:  acc = rnd(acc + rnd(a_ip * b_pj));
 *                     r = rnd(alpha * acc);
 *                     C_ij = (beta == 0) ? r : rnd(r + rnd(beta * C_ij)).
 *   alpha == 0 or k == 0: C_ij = (beta == 0) ? 0 : rnd(beta * C_ij); A and B
 *   are not read.  beta == 0: C is not read (a NaR there is overwritten).
 *   m == 0 or n == 0: nothing is done.
 * Errors: -2/-3 bad trans flag, -4/-5/-6 negative m/n/k, -8/-9 null A or bad
 * lda, -10/-11 null B or bad ldb, -13/-14 null C or bad ldc, -13 also when C
 * aliases A or B (same base pointer); -4 also when m*n needs more than 2^24
 * output tiles of 64 x 32 (one launch).
 */
int posit32_gemm(void* stream, int transa, int transb, int64_t m, int64_t n,
                 int64_t k, posit32_t alpha, const posit32_t* A, int64_t lda,
                 const posit32_t* B, int64_t ldb, posit32_t beta, posit32_t* C,
                 int64_t ldc);

/*
 * Conversions between binary64 and Posit(32,2) (Section 2, Eq. (1)).
 *   posit32_from_f64: out[i] = rnd(x[i]); NaN and +-Inf give NaR, +-0 gives 0.
 *   posit32_to_f64:   out[i] = exact value of p[i]; NaR gives a quiet NaN.
 * n >= 0; x, p, out are device arrays of n elements.  Errors: -2 n < 0,
 * -3/-4 null array with n > 0.
 */
int posit32_from_f64(void* stream, int64_t n, const double* x, posit32_t* out);
int posit32_to_f64(void* stream, int64_t n, const posit32_t* p, double* out);

/*
 * Elementwise arithmetic on device arrays of n elements (the paper's Add,
 * Mul, Div and Sqrt kernels, Section 4.2, Table 2):
 *   op P32_OP_ADD: out = rnd(a + b)      P32_OP_SUB: out = rnd(a - b)
 *   op P32_OP_MUL: out = rnd(a * b)      P32_OP_DIV: out = rnd(a / b), x/0 = NaR
 *   op P32_OP_SQRT: out = rnd(sqrt(a)), b ignored (may be NULL); sqrt of a
 *   negative value is NaR.
 * out may alias a or b.  Errors: -2 bad op, -3 n < 0, -4/-5/-6 null array.
 */
enum { P32_OP_ADD = 0, P32_OP_SUB = 1, P32_OP_MUL = 2, P32_OP_DIV = 3, P32_OP_SQRT = 4 };
int posit32_elementwise(void* stream, int op, int64_t n, const posit32_t* a,
                        const posit32_t* b, posit32_t* out);

/*
 * Blocked factorisations and solves (paper, Section 3: LAPACK's iterative
 * Level-3 LU and Cholesky, MPLAPACK's Rgetrf/Rpotrf, with the solves
 * Rgetrs/Rpotrs of Section 5.1).  Square n x n matrices, row-major, block
 * size 1 <= nb <= 256 (the trailing updates run on posit32_gemm).  The order
 * of every rounded operation (and so every result bit) is fixed:
 *
 * posit32_getrf -- P A = L U with partial pivoting, in place (unit L below the
 *   diagonal, U on and above).  Per panel [j, j+jb): for each column c, the
 *   pivot is argmax_{i>=c} |A[i][c]| in posit order (signed-integer order of
 *   the patterns, |NaR| smallest), ties to the smallest i; rows c and pivot
 *   are swapped inside the panel; A[i][c] = A[i][c] / A[c][c] for i > c
 *   unless the pivot is 0 (then info = c+1 for the first such c and no
 *   scaling); A[i][q] = A[i][q] - rnd(A[i][c]*A[c][q]) for i > c, c < q < j+jb.
 *   Then the interchanges go to the other columns; U12 = L11^-1 A12 column
 *   by column (ascending c); A22 = Rgemm(alpha = -1, beta = 1, L21, U12).
 *   ipiv: device int32[n], 0-based (row c was swapped with row ipiv[c]).
 *   info: device int32[1], 0 or the 1-based column of the first zero pivot
 *   (-1: see below).
 * posit32_getrs -- solve op(A) X = B with the output of posit32_getrf; B is
 *   n x nrhs (ldb >= nrhs), overwritten by X.
 *   op = P32_NOTRANS (A X = B): interchanges in order; forward L (unit): for
 *   c ascending, rows r > c get B[r] - rnd(L[r][c]*B[c]); backward U: for c
 *   descending, B[c] = B[c] / U[c][c], then rows r < c get
 *   B[r] - rnd(U[r][c]*B[c]).
 *   op = P32_TRANS (A^T X = B, LAPACK's trans = 'T'; P A = L U gives
 *   A^T = U^T L^T P): forward U^T: for c ascending, B[c] = B[c] / U[c][c],
 *   rows r > c get B[r] - rnd(U[c][r]*B[c]); backward L^T (unit): for c
 *   descending, rows r < c get B[r] - rnd(L[c][r]*B[c]); then the
 *   interchanges undone in reverse order (c = n-1 .. 0).
 * posit32_potrf -- uplo = P32_LOWER: A = L L^T, in place in the lower
 *   triangle; the strict upper triangle is neither read nor written.
 *   uplo = P32_UPPER: A = U^T U, in place in the upper triangle, the strict
 *   lower triangle neither used nor changed; U is the transpose of the lower
 *   factor of the symmetric matrix held by the upper triangle, bit for bit
 *   (LAPACK's upper variant is the lower one transposed).  The library
 *   exchanges the two strict triangles in place before and after the lower
 *   factorisation (n <= 2^20), so they hold each other's values while the
 *   call runs.  Lower form, per diagonal block:
 *   for each column c: if A[c][c] <= 0 or NaR, info = c+1 and the call stops
 *   (later blocks are not touched); A[c][c] = sqrt(A[c][c]); the block's
 *   rows below are divided by it; the block's lower triangle gets
 *   A[i][q] - rnd(A[i][c]*A[q][c]).  Then L21 = A21 L11^-T row by row
 *   (ascending columns, division by L[c][c]), and the lower triangle of
 *   A22 = Rgemm(-1, 1, L21, L21^T).
 * posit32_potrs -- solve A X = B with the output of posit32_potrf (same
 *   uplo).  Lower: forward L (for c ascending: B[c] = B[c] / L[c][c], rows
 *   below get B[r] - rnd(L[r][c]*B[c])), then backward L^T (for c
 *   descending: B[c] = B[c] / L[c][c], rows above get
 *   B[r] - rnd(L[c][r]*B[c])).  Upper: the same with L[r][c] = U[c][r]
 *   (forward U^T, backward U).
 *
 * All pointers are device memory; calls are stream-ordered and asynchronous
 * (info is written on the device).  posit32_getrf factors each panel in one
 * cooperative launch whose workgroups exchange pivot candidates through a
 * stream-ordered temporary (hipMallocAsync, about 0.5 MB); should that
 * exchange ever wait longer than its bound (a device fault, never a property
 * of the input), info is set to -1.  posit32_potrf takes a stream-ordered
 * temporary of 1 KiB per row (the block column it restores after a failed
 * diagonal).
 * Errors (a negative value is minus the 1-based position of the first bad
 * argument, counting the stream as 1): a bad op / uplo flag; n < 0 (getrf:
 * also n > 2^24 - 2, pivot rows are carried in 24 bits; upper potrf: also
 * n > 2^20); nb outside [1, 256] (getrf/potrf) or nrhs outside
 * [0, 2^31 - 1] (getrs/potrs); a null matrix or lda < max(1, n); then the
 * remaining pointer/leading-dimension arguments in order.
 *
 * Graph capture: posit32_getrs and posit32_potrs launch ordinary kernels
 * only and allocate nothing, so a caller may capture them in a hipGraph
 * (hipStreamBeginCapture on its stream) and replay them, like
 * posit32_gemm, posit32_elementwise, the conversions and the batched calls
 * below.  posit32_getrf (cooperative launches, a stream-ordered temporary)
 * and posit32_potrf (a stream-ordered temporary) are not capturable.
 */
int posit32_getrf(void* stream, int64_t n, int64_t nb, posit32_t* A, int64_t lda,
                  int32_t* ipiv, int32_t* info);
/*
 * posit32_getrf_group -- posit32_getrf on count <= P32_GROUP_MAX independent
 *   square systems at once (the large systems of a serving batch): system i
 *   is n[i] x n[i] at A[i] with leading dimension lda[i], its pivots go to
 *   ipiv[i] and its status to info[i], exactly as posit32_getrf(stream,
 *   n[i], nb, A[i], lda[i], ipiv[i], info[i]) would write them, bit for bit.
 *   The systems advance panel by panel together: at each panel step the
 *   panels of all systems still being factored run in one cooperative launch
 *   (the workgroups split among them by remaining rows), and their
 *   interchanges, U12 solves and trailing updates in one launch each, so the
 *   per-column latency of the panels is shared.  n, A, lda, ipiv and info are
 *   HOST arrays of count entries; the matrices, pivot vectors and info words
 *   they point to are device memory and must not overlap.  Takes a
 *   stream-ordered temporary of about 1 MB + 4 KB per system.  Errors: -2
 *   count outside [0, P32_GROUP_MAX], -3 n NULL or some n[i] outside
 *   [0, 2^24 - 2], -4 nb outside [1, 256], -5 A NULL, A[i] NULL with n[i] >
 *   0, or two systems at one address, -6 lda NULL or lda[i] < max(1, n[i]),
 *   -7 ipiv NULL or ipiv[i] NULL with n[i] > 0, -8 info NULL or info[i] NULL.
 */
#define P32_GROUP_MAX 16
/*
 * posit32_getrs_group -- posit32_getrs (op = P32_NOTRANS) on count <=
 *   P32_GROUP_MAX independent systems at once: system i solves A_i X = B_i
 *   with the factors LU[i] (n[i] x n[i], lda[i]) and pivots ipiv[i] of
 *   posit32_getrf, B[i] n[i] x nrhs[i] with leading dimension ldb[i],
 *   overwritten by X bit for bit as posit32_getrs would.  The substitutions of
 *   all systems advance 64 rows at a time together (one launch per block
 *   step for every system's diagonal block, one for every system's rows
 *   beyond it).  Host arrays of device pointers; nrhs[i] <= 65535; the B[i]
 *   must not overlap.  Allocates nothing.  Errors: -2 count, -3 n, -4 nrhs,
 *   -5 LU, -6 lda, -7 ipiv, -8 B (also two systems sharing one), -9 ldb.
 */
int posit32_getrs_group(void* stream, int count, const int64_t* n, const int64_t* nrhs,
                        const posit32_t* const* LU, const int64_t* lda, const int32_t* const* ipiv,
                        posit32_t* const* B, const int64_t* ldb);
int posit32_getrf_group(void* stream, int count, const int64_t* n, int64_t nb, posit32_t* const* A,
                        const int64_t* lda, int32_t* const* ipiv, int32_t* const* info);

/*
 * posit32_getrf_phases -- a diagnostic: posit32_getrf (same arguments,
 *   validation and result bits), with HIP events recorded between its
 *   launches; returns after the stream has reached the last of them, with
 *   ms[0..3] (HOST memory) the milliseconds spent in the panel
 *   factorisations, the row interchanges outside the panels, the U12 solves
 *   and the trailing updates, summed over the panels.  Errors as
 *   posit32_getrf, -8 ms NULL.
 */
int posit32_getrf_phases(void* stream, int64_t n, int64_t nb, posit32_t* A, int64_t lda,
                         int32_t* ipiv, int32_t* info, double* ms);

/*
 * posit32_getrf_noalloc -- posit32_getrf (same arguments, validation, order
 *   of operations and result bits) for callers that cannot allocate device
 *   memory: code under stream capture by a harness that forbids hipMalloc,
 *   tight serving loops, allocation-free runtimes.  It calls no hipMalloc,
 *   hipMallocAsync, hipFree or other allocating routine: the pivot exchange
 *   uses a file-scope device array of the library (1,056,768 bytes, the
 *   workspace of up to 256 panel workgroups; the call caps each panel at that
 *   many workgroups, so no n that posit32_getrf accepts is refused), which
 *   every GPU the library runs on holds until the process ends.  Its device
 *   address is looked up once per device on the first call (with that device
 *   current); a failure of that lookup is returned as P32_E_HIP - e.  All
 *   calls on one GPU share that GPU's array, and the call sets every word of
 *   it before use: calls that overlap on one GPU (other streams, other host
 *   threads) race on it and must be ordered by the caller.  Like
 *   posit32_getrf it uses cooperative launches and is not capturable.
 */
int posit32_getrf_noalloc(void* stream, int64_t n, int64_t nb, posit32_t* A, int64_t lda,
                          int32_t* ipiv, int32_t* info);
int posit32_getrs(void* stream, int op, int64_t n, int64_t nrhs, const posit32_t* LU,
                  int64_t lda, const int32_t* ipiv, posit32_t* B, int64_t ldb);
int posit32_potrf(void* stream, int uplo, int64_t n, int64_t nb, posit32_t* A, int64_t lda,
                  int32_t* info);
int posit32_potrs(void* stream, int uplo, int64_t n, int64_t nrhs, const posit32_t* L,
                  int64_t lda, posit32_t* B, int64_t ldb);

/*
 * Variable-size batches of the factorisations and solves above: count
 * independent systems in one launch of one workgroup per system (many small
 * systems, the sizes of the paper's LU and Cholesky study, Section 5, in
 * large numbers).
 * Matrix i is factored and solved exactly as the single-matrix call with the
 * same nb would do it, bit for bit.
 *
 *   count        number of systems, 0 <= count <= P32_VBATCH_MAX_COUNT (one
 *                workgroup of 256 threads per system, and a launch counts its
 *                work-items in 32 bits).
 *   max_n        host-side bound, 0 <= n[i] <= max_n <= 2^24 - 2 (a matrix
 *                with a larger n[i] is rejected through its info[i]).
 *   nb           block size, 1 <= nb <= 256.
 *   n, nrhs      device int32[count]: order and right-hand sides of system i.
 *   A (LU, L)    device array of count device pointers to row-major n[i] x
 *                n[i] matrices; lda device int64[count], lda[i] >= max(1, n[i]).
 *   ipiv         device array of count device pointers to int32[n[i]].
 *   B            device array of count device pointers to row-major n[i] x
 *                nrhs[i] matrices; ldb device int64[count], ldb[i] >=
 *                max(1, nrhs[i]).
 *   info         device int32[count], written for every system: 0, or (the
 *                factorisations) the 1-based column of the first zero pivot /
 *                failed diagonal as in the single-matrix calls, or a negative
 *                code for an invalid system, which is then left untouched:
 *                -1 n[i] outside [0, max_n], -2 null A[i] with n[i] > 0,
 *                -3 bad lda[i], -4 null ipiv[i] (LU, n[i] > 0), -5 nrhs[i] < 0,
 *                -6 null B[i] with n[i], nrhs[i] > 0, -7 bad ldb[i].
 * posit32_gesv_vbatched / posit32_posv_vbatched factor and solve in the same
 * launch; a system whose factorisation reports info > 0 is not solved.
 * System i runs in workgroup i, and workgroups start in index order as
 * earlier ones retire, so a batch ordered by decreasing n balances best.  The
 * calls allocate nothing and launch one kernel (they can be captured in a
 * graph).  Systems must not share memory.  Errors: -2 count outside
 * [0, P32_VBATCH_MAX_COUNT], -3 bad max_n, -4 bad nb, -5 a null array
 * argument with count > 0.
 */
#define P32_VBATCH_MAX_COUNT 16777215
int posit32_getrf_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                           posit32_t* const* A, const int64_t* lda, int32_t* const* ipiv,
                           int32_t* info);
int posit32_getrs_vbatched(void* stream, int32_t count, int32_t max_n, const int32_t* n,
                           const int32_t* nrhs, posit32_t* const* LU, const int64_t* lda,
                           int32_t* const* ipiv, posit32_t* const* B, const int64_t* ldb,
                           int32_t* info);
int posit32_gesv_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                          const int32_t* nrhs, posit32_t* const* A, const int64_t* lda,
                          int32_t* const* ipiv, posit32_t* const* B, const int64_t* ldb,
                          int32_t* info);
int posit32_potrf_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                           posit32_t* const* A, const int64_t* lda, int32_t* info);
int posit32_potrs_vbatched(void* stream, int32_t count, int32_t max_n, const int32_t* n,
                           const int32_t* nrhs, posit32_t* const* L, const int64_t* lda,
                           posit32_t* const* B, const int64_t* ldb, int32_t* info);
int posit32_posv_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                          const int32_t* nrhs, posit32_t* const* A, const int64_t* lda,
                          posit32_t* const* B, const int64_t* ldb, int32_t* info);

/*
 * Tuned variable-size batches.  posit32_vbatched runs any of the six batched
 * calls above from one descriptor, with an explicit tuning table; apart from
 * the table nothing changes (same validation, same per-system info, same
 * bits).  The six calls above use the built-in table.
 *
 * The batched kernels factor each panel in sub-panels of `sub` columns (the
 * unblocked pivot search / division / rank-1 updates inside, fused-update
 * chains through the Rgemm tile routine outside; the solves work in blocks of
 * 64 rows, whatever the table).  The width only regroups the work -- every
 * element receives its updates in the unblocked order -- so every table gives
 * the same result bits; it changes only the speed.  A system of order n uses sub[b] of the
 * first bucket b with n <= max_n[b] (the last bucket takes every larger n).
 * paper_2401_14117_amd/autotune.py measures the fastest width per bucket on
 * the device and stores the tables it finds.
 *
 *   posit32_vbatch_tuning: buckets in [1, P32_TUNE_BUCKETS]; max_n strictly
 *     ascending over the used buckets; sub in [1, 64].
 *   posit32_vbatch: kind 0 (LU, as P32_REQ_LU below) or 1 (Cholesky);
 *     factor / solve 0 or 1, at least one set; the other fields as the
 *     arguments of the calls above (ipiv only for LU; nrhs, B, ldb only with
 *     solve; nb only with factor).
 * posit32_vbatched(stream, batch, tuning): tuning NULL = the built-in table
 *   of batch->kind.  Host-side validation only; allocates nothing, one launch
 *   (graph-capturable: the table is copied into the launch arguments).
 *   Errors: -2 batch NULL or any descriptor field invalid (the checks of the
 *   calls above), -3 tuning invalid.
 * posit32_vbatched_default_tuning(kind, out): copies the built-in table of
 *   kind (0 LU, 1 Cholesky) to *out (host memory).  Errors: -1 bad kind,
 *   -2 out NULL.
 */
#define P32_TUNE_BUCKETS 8

typedef struct {
  int32_t buckets;
  int32_t max_n[P32_TUNE_BUCKETS];
  int32_t sub[P32_TUNE_BUCKETS];
} posit32_vbatch_tuning;

typedef struct {
  int32_t kind;              /* 0 LU, 1 Cholesky */
  int32_t factor;            /* 1: factor A */
  int32_t solve;             /* 1: solve with B (after the factorisation, or with given factors) */
  int32_t count;
  int32_t max_n;
  int64_t nb;
  const int32_t* n;
  const int32_t* nrhs;
  posit32_t* const* A;
  const int64_t* lda;
  int32_t* const* ipiv;
  posit32_t* const* B;
  const int64_t* ldb;
  int32_t* info;
} posit32_vbatch;

int posit32_vbatched(void* stream, const posit32_vbatch* batch, const posit32_vbatch_tuning* tuning);
int posit32_vbatched_default_tuning(int kind, posit32_vbatch_tuning* out);

/*
 * Request queue (serving): many independent systems of different sizes,
 * submitted one by one from host memory and solved with continuous batching
 * on the device current at creation.  The queue owns one worker thread, two
 * streams (compute and copy) and a device pool of cfg->device_bytes that holds
 * every admitted system's A, B and pivots and every resident factorisation.
 *
 *  - Admission is in arrival order: a request waits at the head of the queue
 *    until its footprint (4 n^2 + 4 n nrhs + 4 n bytes, each part rounded up
 *    to 256) fits the pool.
 *  - Whenever fewer than two batches are in flight, the worker launches every
 *    admitted waiting request (up to cfg->max_batch) as one batch: systems with
 *    n <= cfg->batch_max_n / 2 through the batched kernels, and those with
 *    n <= cfg->batch_max_n too when at least four of them are in the batch
 *    (alone, such a system is faster through the single-matrix routines);
 *    the others through the single-matrix routines, the new LU systems among
 *    them factored together as by posit32_getrf_group.  Host-to-device copies
 *    overlap the previous batch's computation.
 *  - Each system is factored and solved exactly as posit32_gesv_vbatched /
 *    posit32_posv_vbatched (or the single-matrix calls) with block size
 *    cfg->nb would do it: the solution is bit-identical however requests are
 *    batched.  cfg->tuning (NULL = built-in) points to two sub-panel tables,
 *    [0] for LU and [1] for Cholesky, copied at creation (see
 *    posit32_vbatched).
 *  - keep = 1 keeps a successful factorisation resident; the handle comes
 *    back in posit32_result.factor.  A later request with factor = handle
 *    (same kind and n, A ignored) is solved with it without refactoring.
 *    posit32_factor_release frees it once no request in flight uses it.
 *
 * posit32_queue_submit copies A and B; the caller may reuse them at once.
 * posit32_queue_poll / posit32_queue_wait return 1 while the request is
 * pending; once it has completed they fill *res, copy the n x nrhs solution
 * into X (unless X is NULL), retire the ticket and return res->status: 0, or
 * P32_E_NOMEM (the system can never fit the pool), or a P32_E_HIP code.  info
 * is the factorisation's (as posit32_getrf / posit32_potrf); a factorisation
 * with info > 0 is not solved and not kept (X is then the unsolved B).  Times
 * are seconds on the host's monotonic clock since the queue was created.
 * Back-pressure: with cfg->max_pending > 0, posit32_queue_submit returns
 * P32_E_BUSY (nothing queued) while that many tickets are not yet retired
 * (submitted and not yet returned by a completed poll or wait); the caller
 * collects results and submits again.
 * All calls are thread-safe.  Errors: -1 bad queue or cfg (device_bytes below
 * 1 MiB, max_batch < 1, nb outside 1..256, batch_max_n < 0, max_pending < 0,
 * invalid tuning table), -2 bad request,
 * ticket or factor handle, P32_E_NOMEM from submit for a system larger than
 * the pool.  posit32_queue_destroy finishes every submitted request first.
 */
#define P32_E_NOMEM (-4000)          /* below every P32_E_HIP code */
#define P32_E_BUSY (-5000)           /* submit: cfg->max_pending tickets not yet retired */
enum { P32_REQ_LU = 0, P32_REQ_CHOL = 1 };

typedef struct posit32_queue posit32_queue;

typedef struct {
  int64_t device_bytes;      /* device pool for admitted systems and resident factors */
  int32_t max_batch;         /* most systems per batch */
  int32_t nb;                /* block size of the factorisations */
  int32_t batch_max_n;       /* largest n sent through the batched kernels (see above) */
  const posit32_vbatch_tuning* tuning;   /* NULL, or [LU, Cholesky] tables */
  int64_t max_pending;       /* 0: no limit; else at most this many tickets not yet retired */
} posit32_queue_cfg;

typedef struct {
  int32_t kind;              /* P32_REQ_LU or P32_REQ_CHOL */
  int32_t keep;              /* 1: keep the factorisation resident */
  int64_t n, nrhs;           /* n >= 1, nrhs >= 1 */
  const posit32_t* A;        /* host, n x n row-major (unused with a factor handle) */
  const posit32_t* B;        /* host, n x nrhs row-major */
  uint64_t factor;           /* 0, or a resident factorisation to solve with */
} posit32_request;

typedef struct {
  int32_t status;            /* 1 pending, 0 done, < 0 error */
  int32_t info;
  uint64_t factor;           /* handle of the kept factorisation, else 0 */
  double submit_s, start_s, done_s;
} posit32_result;

typedef struct {
  int64_t pending, inflight_batches, batches, systems_done;
  int64_t pool_bytes, pool_used, resident_factors;
  int32_t error;             /* first runtime failure of the worker, else 0 */
} posit32_queue_stats_t;

int posit32_queue_create(const posit32_queue_cfg* cfg, posit32_queue** q);
int posit32_queue_submit(posit32_queue* q, const posit32_request* req, uint64_t* ticket);
int posit32_queue_poll(posit32_queue* q, uint64_t ticket, posit32_t* X, posit32_result* res);
int posit32_queue_wait(posit32_queue* q, uint64_t ticket, double timeout_s, posit32_t* X,
                       posit32_result* res);
int posit32_factor_release(posit32_queue* q, uint64_t factor);
int posit32_queue_stats(posit32_queue* q, posit32_queue_stats_t* stats);
int posit32_queue_destroy(posit32_queue* q);

#ifdef __cplusplus
}
#endif
#endif /* POSIT32_H */
