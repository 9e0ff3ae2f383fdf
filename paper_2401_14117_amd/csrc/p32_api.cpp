// p32_api.cpp -- the extern "C" boundary of libposit32.so (include/posit32.h):
// host-side argument validation, then a stream-ordered launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "posit32.h"
#include "p32_launch.hpp"

extern "C" {

int posit32_version(void) { return 200; }

const char* posit32_strerror(int code) {
  if (code == 0) return "ok";
  if (code == P32_E_NOMEM) return "the system does not fit the queue's device pool";
  if (code == P32_E_BUSY) return "the queue holds its maximum of unretired requests";
  if (code <= P32_E_HIP) return hipGetErrorString((hipError_t)(P32_E_HIP - code));
  if (code < 0) return "invalid argument (the return value is minus its 1-based position)";
  return "unknown status";
}

int posit32_gemm(void* stream, int transa, int transb, int64_t m, int64_t n, int64_t k,
                 posit32_t alpha, const posit32_t* A, int64_t lda, const posit32_t* B,
                 int64_t ldb, posit32_t beta, posit32_t* C, int64_t ldc) {
  if (transa != P32_NOTRANS && transa != P32_TRANS) return -2;
  if (transb != P32_NOTRANS && transb != P32_TRANS) return -3;
  if (m < 0) return -4;
  if (n < 0) return -5;
  if (k < 0) return -6;
  const int64_t a_width = transa ? m : k;
  const int64_t b_width = transb ? k : n;
  if (lda < (a_width > 1 ? a_width : 1)) return -9;
  if (ldb < (b_width > 1 ? b_width : 1)) return -11;
  if (ldc < (n > 1 ? n : 1)) return -14;
  if (m == 0 || n == 0) return 0;
  if (C == nullptr) return -13;
  const bool reads_ab = alpha != 0u && k > 0;
  if (reads_ab && A == nullptr) return -8;
  if (reads_ab && B == nullptr) return -10;
  if (reads_ab && ((const void*)C == (const void*)A || (const void*)C == (const void*)B)) return -13;
  return p32::launch_gemm((hipStream_t)stream, transa, transb, m, n, k, alpha, A, lda, B, ldb,
                          beta, C, ldc);
}

int posit32_from_f64(void* stream, int64_t n, const double* x, posit32_t* out) {
  if (n < 0) return -2;
  if (n > 0 && x == nullptr) return -3;
  if (n > 0 && out == nullptr) return -4;
  return p32::launch_from_f64((hipStream_t)stream, n, x, out);
}

int posit32_to_f64(void* stream, int64_t n, const posit32_t* p, double* out) {
  if (n < 0) return -2;
  if (n > 0 && p == nullptr) return -3;
  if (n > 0 && out == nullptr) return -4;
  return p32::launch_to_f64((hipStream_t)stream, n, p, out);
}

int posit32_elementwise(void* stream, int op, int64_t n, const posit32_t* a, const posit32_t* b,
                        posit32_t* out) {
  if (op < P32_OP_ADD || op > P32_OP_SQRT) return -2;
  if (n < 0) return -3;
  if (n > 0 && a == nullptr) return -4;
  if (n > 0 && op != P32_OP_SQRT && b == nullptr) return -5;
  if (n > 0 && out == nullptr) return -6;
  return p32::launch_elementwise((hipStream_t)stream, op, n, a, b, out);
}

int posit32_getrf(void* stream, int64_t n, int64_t nb, posit32_t* A, int64_t lda, int32_t* ipiv,
                  int32_t* info) {
  if (n < 0) return -2;
  if (nb < 1 || nb > 256) return -3;
  if (n > 0 && A == nullptr) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > 0 && ipiv == nullptr) return -6;
  if (info == nullptr) return -7;
  if (n > 0xFFFFFE) return -2;                    // pivot rows are carried in 24 bits
  return p32::launch_getrf((hipStream_t)stream, n, nb, A, lda, ipiv, info);
}

int posit32_getrf_group(void* stream, int count, const int64_t* n, int64_t nb, posit32_t* const* A,
                        const int64_t* lda, int32_t* const* ipiv, int32_t* const* info) {
  if (count < 0 || count > P32_GROUP_MAX) return -2;
  if (count == 0) return 0;
  if (n == nullptr) return -3;
  for (int i = 0; i < count; ++i)
    if (n[i] < 0 || n[i] > 0xFFFFFE) return -3;   // pivot rows are carried in 24 bits
  if (nb < 1 || nb > 256) return -4;
  if (A == nullptr) return -5;
  for (int i = 0; i < count; ++i)
    if (n[i] > 0 && A[i] == nullptr) return -5;
  if (lda == nullptr) return -6;
  for (int i = 0; i < count; ++i)
    if (lda[i] < (n[i] > 1 ? n[i] : 1)) return -6;
  if (ipiv == nullptr) return -7;
  for (int i = 0; i < count; ++i)
    if (n[i] > 0 && ipiv[i] == nullptr) return -7;
  if (info == nullptr) return -8;
  for (int i = 0; i < count; ++i)
    if (info[i] == nullptr) return -8;
  for (int i = 0; i < count; ++i)                  // systems must not share memory
    for (int k = 0; k < i; ++k)
      if (n[i] > 0 && n[k] > 0 && A[i] == A[k]) return -5;
  return p32::launch_getrf_group((hipStream_t)stream, count, n, nb, A, lda, ipiv, info);
}

int posit32_getrs_group(void* stream, int count, const int64_t* n, const int64_t* nrhs, const posit32_t* const* LU,
                        const int64_t* lda, const int32_t* const* ipiv, posit32_t* const* B, const int64_t* ldb) {
  if (count < 0 || count > P32_GROUP_MAX) return -2;
  if (count == 0) return 0;
  if (n == nullptr) return -3;
  for (int i = 0; i < count; ++i)
    if (n[i] < 0) return -3;
  if (nrhs == nullptr) return -4;
  for (int i = 0; i < count; ++i)
    if (nrhs[i] < 0 || nrhs[i] > 65535) return -4;
  if (LU == nullptr) return -5;
  for (int i = 0; i < count; ++i)
    if (n[i] > 0 && LU[i] == nullptr) return -5;
  if (lda == nullptr) return -6;
  for (int i = 0; i < count; ++i)
    if (lda[i] < (n[i] > 1 ? n[i] : 1)) return -6;
  if (ipiv == nullptr) return -7;
  for (int i = 0; i < count; ++i)
    if (n[i] > 0 && ipiv[i] == nullptr) return -7;
  if (B == nullptr) return -8;
  for (int i = 0; i < count; ++i)
    if (n[i] > 0 && nrhs[i] > 0 && B[i] == nullptr) return -8;
  if (ldb == nullptr) return -9;
  for (int i = 0; i < count; ++i)
    if (ldb[i] < (nrhs[i] > 1 ? nrhs[i] : 1)) return -9;
  for (int i = 0; i < count; ++i)                  // right-hand sides must not be shared
    for (int k = 0; k < i; ++k)
      if (n[i] > 0 && nrhs[i] > 0 && n[k] > 0 && nrhs[k] > 0 && B[i] == B[k]) return -8;
  return p32::launch_getrs_group((hipStream_t)stream, count, n, nrhs, LU, lda, ipiv, B, ldb);
}

int posit32_getrf_phases(void* stream, int64_t n, int64_t nb, posit32_t* A, int64_t lda, int32_t* ipiv,
                         int32_t* info, double* ms) {
  if (n < 0) return -2;
  if (nb < 1 || nb > 256) return -3;
  if (n > 0 && A == nullptr) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > 0 && ipiv == nullptr) return -6;
  if (info == nullptr) return -7;
  if (ms == nullptr) return -8;
  if (n > 0xFFFFFE) return -2;
  return p32::launch_getrf_phases((hipStream_t)stream, n, nb, A, lda, ipiv, info, ms);
}

int posit32_getrf_noalloc(void* stream, int64_t n, int64_t nb, posit32_t* A, int64_t lda,
                          int32_t* ipiv, int32_t* info) {
  if (n < 0) return -2;
  if (nb < 1 || nb > 256) return -3;
  if (n > 0 && A == nullptr) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > 0 && ipiv == nullptr) return -6;
  if (info == nullptr) return -7;
  if (n > 0xFFFFFE) return -2;                    // pivot rows are carried in 24 bits
  return p32::launch_getrf_noalloc((hipStream_t)stream, n, nb, A, lda, ipiv, info);
}

int posit32_getrs(void* stream, int op, int64_t n, int64_t nrhs, const posit32_t* LU, int64_t lda,
                  const int32_t* ipiv, posit32_t* B, int64_t ldb) {
  if (op != P32_NOTRANS && op != P32_TRANS) return -2;
  if (n < 0) return -3;
  if (nrhs < 0 || nrhs > 0x7FFFFFFF) return -4;   // one workgroup per right-hand side
  if (n > 0 && LU == nullptr) return -5;
  if (lda < (n > 1 ? n : 1)) return -6;
  if (n > 0 && ipiv == nullptr) return -7;
  if (n > 0 && nrhs > 0 && B == nullptr) return -8;
  if (ldb < (nrhs > 1 ? nrhs : 1)) return -9;
  return p32::launch_getrs((hipStream_t)stream, op, n, nrhs, LU, lda, ipiv, B, ldb);
}

int posit32_potrf(void* stream, int uplo, int64_t n, int64_t nb, posit32_t* A, int64_t lda,
                  int32_t* info) {
  if (uplo != P32_LOWER && uplo != P32_UPPER) return -2;
  if (n < 0) return -3;
  if (nb < 1 || nb > 256) return -4;
  if (n > 0 && A == nullptr) return -5;
  if (lda < (n > 1 ? n : 1)) return -6;
  if (info == nullptr) return -7;
  if (uplo == P32_UPPER && n > ((int64_t)1 << 20)) return -3;   // triangle exchange: one launch
  return p32::launch_potrf((hipStream_t)stream, uplo, n, nb, A, lda, info);
}

int posit32_potrs(void* stream, int uplo, int64_t n, int64_t nrhs, const posit32_t* L, int64_t lda,
                  posit32_t* B, int64_t ldb) {
  if (uplo != P32_LOWER && uplo != P32_UPPER) return -2;
  if (n < 0) return -3;
  if (nrhs < 0 || nrhs > 0x7FFFFFFF) return -4;
  if (n > 0 && L == nullptr) return -5;
  if (lda < (n > 1 ? n : 1)) return -6;
  if (n > 0 && nrhs > 0 && B == nullptr) return -7;
  if (ldb < (nrhs > 1 ? nrhs : 1)) return -8;
  return p32::launch_potrs((hipStream_t)stream, uplo, n, nrhs, L, lda, B, ldb);
}

// ---- variable-size batches ---------------------------------------------------

static int vb_common(int32_t count, int32_t max_n, const int32_t* n, posit32_t* const* A,
                     const int64_t* lda, int32_t* info) {
  if (count < 0 || count > P32_VBATCH_MAX_COUNT) return -2;
  if (max_n < 0 || max_n > 0xFFFFFE) return -3;
  if (count > 0 && (n == nullptr || A == nullptr || lda == nullptr || info == nullptr)) return -5;
  return 0;
}

int posit32_getrf_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                           posit32_t* const* A, const int64_t* lda, int32_t* const* ipiv,
                           int32_t* info) {
  const int rc = vb_common(count, max_n, n, A, lda, info);
  if (rc) return rc;
  if (nb < 1 || nb > 256) return -4;
  if (count > 0 && ipiv == nullptr) return -5;
  return p32::launch_vbatched((hipStream_t)stream, 0, true, false, count, max_n, nb, n, A, lda, ipiv,
                              nullptr, nullptr, nullptr, info);
}

int posit32_getrs_vbatched(void* stream, int32_t count, int32_t max_n, const int32_t* n,
                           const int32_t* nrhs, posit32_t* const* LU, const int64_t* lda,
                           int32_t* const* ipiv, posit32_t* const* B, const int64_t* ldb,
                           int32_t* info) {
  const int rc = vb_common(count, max_n, n, LU, lda, info);
  if (rc) return rc;
  if (count > 0 && (nrhs == nullptr || ipiv == nullptr || B == nullptr || ldb == nullptr)) return -5;
  return p32::launch_vbatched((hipStream_t)stream, 0, false, true, count, max_n, 1, n, LU, lda, ipiv,
                              nrhs, B, ldb, info);
}

int posit32_gesv_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                          const int32_t* nrhs, posit32_t* const* A, const int64_t* lda,
                          int32_t* const* ipiv, posit32_t* const* B, const int64_t* ldb,
                          int32_t* info) {
  const int rc = vb_common(count, max_n, n, A, lda, info);
  if (rc) return rc;
  if (nb < 1 || nb > 256) return -4;
  if (count > 0 && (nrhs == nullptr || ipiv == nullptr || B == nullptr || ldb == nullptr)) return -5;
  return p32::launch_vbatched((hipStream_t)stream, 0, true, true, count, max_n, nb, n, A, lda, ipiv,
                              nrhs, B, ldb, info);
}

int posit32_potrf_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                           posit32_t* const* A, const int64_t* lda, int32_t* info) {
  const int rc = vb_common(count, max_n, n, A, lda, info);
  if (rc) return rc;
  if (nb < 1 || nb > 256) return -4;
  return p32::launch_vbatched((hipStream_t)stream, 1, true, false, count, max_n, nb, n, A, lda, nullptr,
                              nullptr, nullptr, nullptr, info);
}

int posit32_potrs_vbatched(void* stream, int32_t count, int32_t max_n, const int32_t* n,
                           const int32_t* nrhs, posit32_t* const* L, const int64_t* lda,
                           posit32_t* const* B, const int64_t* ldb, int32_t* info) {
  const int rc = vb_common(count, max_n, n, L, lda, info);
  if (rc) return rc;
  if (count > 0 && (nrhs == nullptr || B == nullptr || ldb == nullptr)) return -5;
  return p32::launch_vbatched((hipStream_t)stream, 1, false, true, count, max_n, 1, n, L, lda, nullptr,
                              nrhs, B, ldb, info);
}

int posit32_posv_vbatched(void* stream, int32_t count, int32_t max_n, int64_t nb, const int32_t* n,
                          const int32_t* nrhs, posit32_t* const* A, const int64_t* lda,
                          posit32_t* const* B, const int64_t* ldb, int32_t* info) {
  const int rc = vb_common(count, max_n, n, A, lda, info);
  if (rc) return rc;
  if (nb < 1 || nb > 256) return -4;
  if (count > 0 && (nrhs == nullptr || B == nullptr || ldb == nullptr)) return -5;
  return p32::launch_vbatched((hipStream_t)stream, 1, true, true, count, max_n, nb, n, A, lda, nullptr,
                              nrhs, B, ldb, info);
}

static bool tuning_ok(const posit32_vbatch_tuning& t) {
  if (t.buckets < 1 || t.buckets > P32_TUNE_BUCKETS) return false;
  for (int b = 0; b < t.buckets; ++b) {
    if (t.sub[b] < 1 || t.sub[b] > 64) return false;
    if (b > 0 && t.max_n[b] <= t.max_n[b - 1]) return false;
  }
  return true;
}

static p32::Tuning to_tuning(const posit32_vbatch_tuning& t) {
  p32::Tuning r{};
  static_assert(p32::kTuneBuckets == P32_TUNE_BUCKETS, "bucket count of the C ABI and the kernels");
  r.buckets = t.buckets;
  for (int b = 0; b < P32_TUNE_BUCKETS; ++b) {
    r.max_n[b] = t.max_n[b];
    r.sub[b] = t.sub[b];
  }
  return r;
}

int posit32_vbatched(void* stream, const posit32_vbatch* bt, const posit32_vbatch_tuning* tuning) {
  if (bt == nullptr) return -2;
  if (bt->kind != 0 && bt->kind != 1) return -2;
  if ((bt->factor != 0 && bt->factor != 1) || (bt->solve != 0 && bt->solve != 1)) return -2;
  if (!bt->factor && !bt->solve) return -2;
  if (vb_common(bt->count, bt->max_n, bt->n, bt->A, bt->lda, bt->info)) return -2;
  if (bt->factor && (bt->nb < 1 || bt->nb > 256)) return -2;
  if (bt->count > 0 && bt->kind == 0 && bt->ipiv == nullptr) return -2;
  if (bt->count > 0 && bt->solve && (bt->nrhs == nullptr || bt->B == nullptr || bt->ldb == nullptr))
    return -2;
  p32::Tuning t{};
  if (tuning != nullptr) {
    if (!tuning_ok(*tuning)) return -3;
    t = to_tuning(*tuning);
  } else {
    t = p32::default_tuning(bt->kind);
  }
  return p32::launch_vbatched((hipStream_t)stream, bt->kind, bt->factor != 0, bt->solve != 0, bt->count,
                              bt->max_n, bt->factor ? bt->nb : 1, bt->n, bt->A, bt->lda,
                              bt->kind == 0 ? bt->ipiv : nullptr, bt->solve ? bt->nrhs : nullptr,
                              bt->solve ? bt->B : nullptr, bt->solve ? bt->ldb : nullptr, bt->info, &t);
}

int posit32_vbatched_default_tuning(int kind, posit32_vbatch_tuning* out) {
  if (kind != 0 && kind != 1) return -1;
  if (out == nullptr) return -2;
  const p32::Tuning t = p32::default_tuning(kind);
  *out = posit32_vbatch_tuning{};
  out->buckets = t.buckets;
  for (int b = 0; b < P32_TUNE_BUCKETS; ++b) {
    out->max_n[b] = t.max_n[b];
    out->sub[b] = t.sub[b];
  }
  return 0;
}

}  // extern "C"

int p32::tuning_from_abi(const posit32_vbatch_tuning& t, p32::Tuning* out) {
  if (!tuning_ok(t)) return -1;
  *out = to_tuning(t);
  return 0;
}
