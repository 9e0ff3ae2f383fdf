/*
 * ref_lapack.c -- reference blocked LU and Cholesky factorisations and
 * solves in Posit(32,2).  TEST INFRASTRUCTURE ONLY (see posit_oracle.h):
 * plain loops in the order stated below, every product and sum rounded by
 * the oracle's own arithmetic.
 *
 * The paper factors with LAPACK's iterative (right-looking, blocked)
 * algorithms in which only the trailing update calls Rgemm (Section 3,
 * Section 5.2).  It gives no block size and no order for the unblocked
 * parts; the order used here, block size nb, is:
 *
 * Rgetrf (partial pivoting), for each panel of columns [j, j+jb):
 *   1. for c = j .. j+jb-1 (column by column inside the panel):
 *        pivot p = argmax_{i >= c} |A[i][c]| in posit order (the signed
 *        integer order of the patterns; |NaR| = NaR is the smallest),
 *        ties to the smallest i; ipiv[c] = p; swap rows c and p inside the
 *        panel; if A[c][c] != 0: A[i][c] = A[i][c] / A[c][c] for i > c,
 *        else info = c+1 (first such c) and no scaling; then for i > c and
 *        q in (c, j+jb): A[i][q] = A[i][q] - rnd(A[i][c] * A[c][q]).
 *   2. apply the panel's interchanges, in order, to the columns outside it;
 *   3. U12 = L11^-1 A12 (unit lower): for c ascending, for r in (c, j+jb):
 *        A[r][q] = A[r][q] - rnd(A[r][c] * A[c][q]) for the columns right of
 *        the panel;
 *   4. A22 = Rgemm(alpha = -1, beta = 1, L21, U12) with k = jb.
 * Rgetrs: apply ipiv in order; forward L (unit): for c ascending, rows r > c
 *   get b[r] - rnd(L[r][c] * b[c]); backward U: for c descending,
 *   b[c] = b[c] / U[c][c], then rows r < c get b[r] - rnd(U[r][c] * b[c]).
 * Rpotrf (lower), for each diagonal block [j, j+jb):
 *   1. for c in the block: if A[c][c] <= 0 or NaR: info = c+1, stop;
 *        d = sqrt(A[c][c]); A[c][c] = d; A[i][c] = A[i][c] / d for i > c in
 *        the block; then A[i][q] = A[i][q] - rnd(A[i][c] * A[q][c]) for
 *        c < q <= i in the block;
 *   2. L21 = A21 L11^-T row by row: for c ascending, x = A[r][c], then
 *        x = x - rnd(A[r][q] * L[c][q]) for q = j..c-1 ascending,
 *        A[r][c] = x / L[c][c];
 *   3. lower triangle of A22 = Rgemm(alpha = -1, beta = 1, L21, L21^T).
 * Rpotrs: forward L: for c ascending, b[c] = b[c] / L[c][c], rows r > c get
 *   b[r] - rnd(L[r][c] * b[c]); backward L^T: for c descending,
 *   b[c] = b[c] / L[c][c], rows r < c get b[r] - rnd(L[c][r] * b[c]).
 * Only the lower triangle of A is referenced or written by Rpotrf/Rpotrs.
 *
 * The transposed and upper forms (LAPACK's trans = 'T' and uplo = 'U'):
 * Rgetrs with op = T solves A^T X = B.  P A = L U gives A^T = U^T L^T P, so:
 *   forward U^T: for c ascending, b[c] = b[c] / U[c][c], rows r > c get
 *   b[r] - rnd(U[c][r] * b[c]); backward L^T (unit): for c descending, rows
 *   r < c get b[r] - rnd(L[c][r] * b[c]); then the interchanges in reverse
 *   order (c = n-1 .. 0).
 * Rpotrf, upper: A = U^T U with U in the upper triangle.  The upper variant
 *   is the lower one transposed: U^T is the lower factor, by the schedule
 *   above, of the symmetric matrix whose lower triangle is the transpose of
 *   A's upper triangle.  The strict lower triangle of A is neither read nor
 *   written; a failed diagonal leaves the same partial state, transposed.
 * Rpotrs, upper: forward U^T: for c ascending, b[c] = b[c] / U[c][c], rows
 *   r > c get b[r] - rnd(U[c][r] * b[c]); backward U: for c descending,
 *   b[c] = b[c] / U[c][c], rows r < c get b[r] - rnd(U[r][c] * b[c]).
 */
#include <stdlib.h>
#include <stdint.h>

#include "posit_oracle.h"

#define NAR 0x80000000u
#define ONE 0x40000000u
#define MINUS_ONE 0xC0000000u

static uint32_t padd(uint32_t a, uint32_t b) { return oracle_posit_add(32, a, b); }
static uint32_t pmul(uint32_t a, uint32_t b) { return oracle_posit_mul(32, a, b); }
static uint32_t pdiv(uint32_t a, uint32_t b) { return oracle_posit_div(32, a, b); }
static uint32_t psqrt(uint32_t a) { return oracle_posit_sqrt(32, a); }
static uint32_t pneg(uint32_t a) { return 0u - a; }

/* a - rnd(b * c) */
static uint32_t pfms(uint32_t a, uint32_t b, uint32_t c) { return padd(a, pneg(pmul(b, c))); }

/* key of |x| in posit order */
static int32_t abs_key(uint32_t x) {
  if (x == NAR) return INT32_MIN;
  const int32_t s = (int32_t)x;
  return s < 0 ? -s : s;
}

static void swap_rows(uint32_t* A, int64_t lda, int64_t r1, int64_t r2, int64_t c0, int64_t c1) {
  for (int64_t q = c0; q < c1; ++q) {
    const uint32_t t = A[r1 * lda + q];
    A[r1 * lda + q] = A[r2 * lda + q];
    A[r2 * lda + q] = t;
  }
}

void oracle_getrf(int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* ipiv, int32_t* info) {
  *info = 0;
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    /* 1. panel */
    for (int64_t c = j; c < j + jb; ++c) {
      int64_t p = c;
      int32_t best = abs_key(A[c * lda + c]);
      for (int64_t i = c + 1; i < n; ++i) {
        const int32_t key = abs_key(A[i * lda + c]);
        if (key > best) { best = key; p = i; }
      }
      ipiv[c] = (int32_t)p;
      if (p != c) swap_rows(A, lda, c, p, j, j + jb);
      const uint32_t piv = A[c * lda + c];
      if (piv == 0u) {
        if (*info == 0) *info = (int32_t)(c + 1);
      } else {
        for (int64_t i = c + 1; i < n; ++i) A[i * lda + c] = pdiv(A[i * lda + c], piv);
      }
#pragma omp parallel for schedule(static)
      for (int64_t i = c + 1; i < n; ++i)
        for (int64_t q = c + 1; q < j + jb; ++q)
          A[i * lda + q] = pfms(A[i * lda + q], A[i * lda + c], A[c * lda + q]);
    }
    /* 2. interchanges outside the panel */
    for (int64_t c = j; c < j + jb; ++c) {
      const int64_t p = ipiv[c];
      if (p != c) {
        swap_rows(A, lda, c, p, 0, j);
        swap_rows(A, lda, c, p, j + jb, n);
      }
    }
    if (j + jb < n) {
      /* 3. U12 = L11^-1 A12 */
#pragma omp parallel for schedule(static)
      for (int64_t q = j + jb; q < n; ++q)          /* columns are independent */
        for (int64_t c = j; c < j + jb; ++c)
          for (int64_t r = c + 1; r < j + jb; ++r)
            A[r * lda + q] = pfms(A[r * lda + q], A[r * lda + c], A[c * lda + q]);
      /* 4. trailing update */
      const int64_t mm = n - j - jb;
      oracle_gemm(0, 0, mm, mm, jb, MINUS_ONE, &A[(j + jb) * lda + j], lda,
                  &A[j * lda + j + jb], lda, ONE, &A[(j + jb) * lda + j + jb], lda);
    }
  }
}

void oracle_getrs(int64_t n, int64_t nrhs, const uint32_t* LU, int64_t lda, const int32_t* ipiv,
                  uint32_t* B, int64_t ldb) {
  for (int64_t c = 0; c < n; ++c)
    if (ipiv[c] != c) swap_rows(B, ldb, c, ipiv[c], 0, nrhs);
  for (int64_t c = 0; c < n; ++c)
    for (int64_t r = c + 1; r < n; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], LU[r * lda + c], B[c * ldb + q]);
  for (int64_t c = n - 1; c >= 0; --c) {
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], LU[c * lda + c]);
    for (int64_t r = 0; r < c; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], LU[r * lda + c], B[c * ldb + q]);
  }
}

void oracle_potrf(int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info) {
  *info = 0;
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t jb = nb < n - j ? nb : n - j;
    /* 1. diagonal block */
    for (int64_t c = j; c < j + jb; ++c) {
      const uint32_t a = A[c * lda + c];
      if ((int32_t)a <= 0) {            /* non-positive, or NaR */
        *info = (int32_t)(c + 1);
        return;
      }
      const uint32_t d = psqrt(a);
      A[c * lda + c] = d;
      for (int64_t i = c + 1; i < j + jb; ++i) A[i * lda + c] = pdiv(A[i * lda + c], d);
      for (int64_t i = c + 1; i < j + jb; ++i)
        for (int64_t q = c + 1; q <= i; ++q)
          A[i * lda + q] = pfms(A[i * lda + q], A[i * lda + c], A[q * lda + c]);
    }
    if (j + jb < n) {
      /* 2. L21 = A21 L11^-T */
#pragma omp parallel for schedule(static)
      for (int64_t r = j + jb; r < n; ++r)
        for (int64_t c = j; c < j + jb; ++c) {
          uint32_t x = A[r * lda + c];
          for (int64_t q = j; q < c; ++q) x = pfms(x, A[r * lda + q], A[c * lda + q]);
          A[r * lda + c] = pdiv(x, A[c * lda + c]);
        }
      /* 3. lower triangle of A22 = Rgemm(-1, 1, L21, L21^T) */
#pragma omp parallel for schedule(dynamic, 1)
      for (int64_t i = j + jb; i < n; ++i)
        for (int64_t q = j + jb; q <= i; ++q) {
          uint32_t acc = 0;
          for (int64_t p = j; p < j + jb; ++p)
            acc = padd(acc, pmul(A[i * lda + p], A[q * lda + p]));
          const uint32_t r = pmul(MINUS_ONE, acc);
          A[i * lda + q] = padd(r, pmul(ONE, A[i * lda + q]));
        }
    }
  }
}

void oracle_potrs(int64_t n, int64_t nrhs, const uint32_t* L, int64_t lda, uint32_t* B,
                  int64_t ldb) {
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], L[c * lda + c]);
    for (int64_t r = c + 1; r < n; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], L[r * lda + c], B[c * ldb + q]);
  }
  for (int64_t c = n - 1; c >= 0; --c) {
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], L[c * lda + c]);
    for (int64_t r = 0; r < c; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], L[c * lda + r], B[c * ldb + q]);
  }
}

void oracle_getrs_trans(int64_t n, int64_t nrhs, const uint32_t* LU, int64_t lda,
                        const int32_t* ipiv, uint32_t* B, int64_t ldb) {
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], LU[c * lda + c]);
    for (int64_t r = c + 1; r < n; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], LU[c * lda + r], B[c * ldb + q]);
  }
  for (int64_t c = n - 1; c >= 0; --c)
    for (int64_t r = 0; r < c; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], LU[c * lda + r], B[c * ldb + q]);
  for (int64_t c = n - 1; c >= 0; --c)
    if (ipiv[c] != c) swap_rows(B, ldb, c, ipiv[c], 0, nrhs);
}

/* returns 0, or -1 when the transposed copy cannot be allocated */
int oracle_potrf_upper(int64_t n, int64_t nb, uint32_t* A, int64_t lda, int32_t* info) {
  *info = 0;
  if (n == 0) return 0;
  uint32_t* T = (uint32_t*)malloc((size_t)n * (size_t)n * sizeof(uint32_t));
  if (T == NULL) return -1;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) T[i * n + j] = j <= i ? A[j * lda + i] : 0u;
  oracle_potrf(n, nb, T, n, info);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) A[j * lda + i] = T[i * n + j];
  free(T);
  return 0;
}

void oracle_potrs_upper(int64_t n, int64_t nrhs, const uint32_t* U, int64_t lda, uint32_t* B,
                        int64_t ldb) {
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], U[c * lda + c]);
    for (int64_t r = c + 1; r < n; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], U[c * lda + r], B[c * ldb + q]);
  }
  for (int64_t c = n - 1; c >= 0; --c) {
    for (int64_t q = 0; q < nrhs; ++q) B[c * ldb + q] = pdiv(B[c * ldb + q], U[c * lda + c]);
    for (int64_t r = 0; r < c; ++r)
      for (int64_t q = 0; q < nrhs; ++q)
        B[r * ldb + q] = pfms(B[r * ldb + q], U[r * lda + c], B[c * ldb + q]);
  }
}
