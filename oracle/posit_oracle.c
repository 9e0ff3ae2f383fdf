/*
 * posit_oracle.c -- reference Posit(N,2) arithmetic and reference Rgemm.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle the GPU library is checked
 * against: a plain, slow, obviously correct CPU implementation written from
 * the definition of the format (paper, Section 2, Eq. (1)).  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Method.  Every operand is decoded bit by bit into an exact value held as a
 * wide sign-magnitude fixed-point number (bit i has weight 2^(i-XLSB)).  The
 * exact sum or product is formed in that representation; quotients and square
 * roots are formed with enough extra bits plus a sticky flag.  The exact value
 * is then rounded by writing out its infinitely precise posit bit string
 * (regime run, terminator, two exponent bits, fraction bits) and rounding that
 * string to N-1 bits after the sign, to nearest with ties to the even pattern.
 * Values at or beyond maxpos give maxpos, values at or below minpos give
 * minpos; a nonzero value never rounds to 0 or NaR.  (The paper states only
 * that the fraction is rounded at the new fraction length, Section 2; this is
 * the rounding of the posit standard that SoftPosit, which the paper ports,
 * implements.)
 */
#include "posit_oracle.h"

#include <assert.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Exact values                                                              */
/* ------------------------------------------------------------------------ */

#define XLIMBS 20            /* 640-bit magnitude                           */
#define XBITS (32 * XLIMBS)
#define XLSB 320             /* bit XLSB has weight 2^0                      */

typedef struct {
  int neg;                   /* sign of the value                           */
  uint32_t w[XLIMBS];        /* magnitude, little-endian 32-bit limbs       */
  int sticky;                /* true magnitude is above w by less than one
                                unit of bit 0 (inexact quotients / roots)   */
} xnum;

static void x_zero(xnum* x) { memset(x, 0, sizeof *x); }

static int x_bit(const xnum* x, int i) {
  if (i < 0 || i >= XBITS) return 0;
  return (int)((x->w[i >> 5] >> (i & 31)) & 1u);
}

static int x_top(const xnum* x) {        /* index of highest set bit, or -1 */
  for (int l = XLIMBS - 1; l >= 0; --l)
    if (x->w[l]) return 32 * l + 31 - __builtin_clz(x->w[l]);
  return -1;
}

static int x_any_below(const xnum* x, int i) {  /* any bit with index < i */
  if (i <= 0) return 0;
  if (i > XBITS) i = XBITS;
  int l = i >> 5, r = i & 31;
  for (int j = 0; j < l; ++j)
    if (x->w[j]) return 1;
  if (r && (x->w[l] & ((1u << r) - 1u))) return 1;
  return 0;
}

/* magnitude += v * 2^(bit index pos) */
static void x_add_u128_at(xnum* x, unsigned __int128 v, int pos) {
  assert(pos >= 0);
  for (int b = 0; v != 0; ++b, v >>= 1) {
    if (!(v & 1)) continue;
    int i = pos + b;
    assert(i < XBITS);
    /* add 2^i with carry propagation */
    int l = i >> 5;
    uint64_t add = (uint64_t)1 << (i & 31);
    while (add && l < XLIMBS) {
      uint64_t s = (uint64_t)x->w[l] + add;
      x->w[l] = (uint32_t)s;
      add = s >> 32;
      ++l;
    }
    assert(add == 0);
  }
}

static int x_cmpmag(const xnum* a, const xnum* b) {
  for (int l = XLIMBS - 1; l >= 0; --l) {
    if (a->w[l] > b->w[l]) return 1;
    if (a->w[l] < b->w[l]) return -1;
  }
  return 0;
}

/* exact a + b (both exact: no sticky) */
static xnum x_add(const xnum* a, const xnum* b) {
  assert(!a->sticky && !b->sticky);
  xnum r;
  x_zero(&r);
  if (a->neg == b->neg) {
    uint64_t c = 0;
    for (int l = 0; l < XLIMBS; ++l) {
      uint64_t s = (uint64_t)a->w[l] + b->w[l] + c;
      r.w[l] = (uint32_t)s;
      c = s >> 32;
    }
    assert(c == 0);
    r.neg = a->neg;
  } else {
    int c = x_cmpmag(a, b);
    if (c == 0) return r;                 /* exact cancellation gives +0 */
    const xnum* big = c > 0 ? a : b;
    const xnum* sml = c > 0 ? b : a;
    int64_t borrow = 0;
    for (int l = 0; l < XLIMBS; ++l) {
      int64_t d = (int64_t)big->w[l] - (int64_t)sml->w[l] - borrow;
      borrow = d < 0;
      r.w[l] = (uint32_t)(d + (borrow ? ((int64_t)1 << 32) : 0));
    }
    assert(borrow == 0);
    r.neg = big->neg;
  }
  return r;
}

/* ------------------------------------------------------------------------ */
/* Decoding (Section 2, Eq. (1))                                             */
/* ------------------------------------------------------------------------ */

enum { P_NORMAL = 0, P_ZERO = 1, P_NAR = 2 };

typedef struct {
  int kind;
  int neg;
  int k;          /* regime value                                           */
  int e;          /* exponent bits (missing bits read as 0)                 */
  int fs;         /* number of fraction bits present                        */
  uint32_t f;     /* fraction bits                                          */
} pdec;

static uint32_t pmask(int N) { return N == 32 ? 0xFFFFFFFFu : ((1u << N) - 1u); }
static uint32_t p_nar(int N) { return 1u << (N - 1); }
static uint32_t p_maxpos(int N) { return (1u << (N - 1)) - 1u; }
static int p_maxscale(int N) { return 4 * (N - 2); }  /* maxpos = 16^(N-2) */

static pdec p_decode(int N, uint32_t p) {
  pdec d;
  memset(&d, 0, sizeof d);
  p &= pmask(N);
  if (p == 0) { d.kind = P_ZERO; return d; }
  if (p == p_nar(N)) { d.kind = P_NAR; return d; }
  d.kind = P_NORMAL;
  d.neg = (int)((p >> (N - 1)) & 1u);
  uint32_t a = d.neg ? ((0u - p) & pmask(N)) : p;      /* pattern of |x| */
  int i = N - 2;                                       /* bit after sign */
  int r0 = (int)((a >> i) & 1u);
  int m = 0;                                           /* run length     */
  while (i >= 0 && (int)((a >> i) & 1u) == r0) { ++m; --i; }
  d.k = r0 ? m - 1 : -m;
  --i;                                                 /* terminator     */
  int e = 0;
  for (int j = 0; j < 2; ++j) {
    e <<= 1;
    if (i >= 0) { e |= (int)((a >> i) & 1u); --i; }
  }
  d.e = e;
  d.fs = i + 1 > 0 ? i + 1 : 0;
  d.f = d.fs ? (a & ((1u << d.fs) - 1u)) : 0u;
  return d;
}

/* significand (1.f as an integer) and the weight of its last bit */
static uint64_t p_sig(const pdec* d) { return ((uint64_t)1 << d->fs) + d->f; }
static int p_lsbexp(const pdec* d) { return 4 * d->k + d->e - d->fs; }

static xnum x_from_dec(const pdec* d) {
  xnum x;
  x_zero(&x);
  if (d->kind != P_NORMAL) return x;
  x.neg = d->neg;
  x_add_u128_at(&x, p_sig(d), p_lsbexp(d) + XLSB);
  return x;
}

/* ------------------------------------------------------------------------ */
/* Rounding an exact value to Posit(N,2)                                     */
/* ------------------------------------------------------------------------ */

static int floor_div4(int v) { return v >= 0 ? v / 4 : -((-v + 3) / 4); }

/* bit j (0 = first bit after the sign) of the infinitely precise posit string
   of a value whose leading magnitude bit is t, with regime k, exponent e and
   regime length R (run plus terminator) */
static int strbit(const xnum* x, int t, int k, int e, int R, int j) {
  if (j < R - 1) return k >= 0 ? 1 : 0;          /* regime run         */
  if (j == R - 1) return k >= 0 ? 0 : 1;         /* terminator         */
  if (j == R) return (e >> 1) & 1;               /* exponent, high bit */
  if (j == R + 1) return e & 1;                  /* exponent, low bit  */
  return x_bit(x, t - 1 - (j - R - 2));          /* fraction bits      */
}

static uint32_t x_round(int N, const xnum* x) {
  int t = x_top(x);
  uint32_t P;
  if (t < 0 && !x->sticky) return 0;
  int maxsc = p_maxscale(N);
  int sc = t - XLSB;                             /* floor(log2 |x|)    */
  if (t < 0) {
    P = 1u;                                      /* below bit 0: tiny  */
  } else if (sc >= maxsc) {
    P = p_maxpos(N);                             /* |x| >= maxpos      */
  } else if (sc < -maxsc ||
             (sc == -maxsc && !x_any_below(x, t) && !x->sticky)) {
    P = 1u;                                      /* |x| <= minpos      */
  } else {
    int k = floor_div4(sc);
    int e = sc - 4 * k;
    int R = k >= 0 ? k + 2 : -k + 1;
    P = 0;
    for (int j = 0; j < N - 1; ++j) P = (P << 1) | (uint32_t)strbit(x, t, k, e, R, j);
    int G = strbit(x, t, k, e, R, N - 1);
    int S = x->sticky;
    for (int j = N; j < R + 2; ++j) S |= strbit(x, t, k, e, R, j);
    int j0 = N > R + 2 ? N : R + 2;   /* first later string bit that is a
                                          fraction bit                      */
    int i0 = t - 1 - (j0 - R - 2);    /* its magnitude bit index           */
    S |= x_any_below(x, i0 + 1);
    if (G && (S || (P & 1u))) P += 1u;
  }
  if (x->neg) P = (0u - P) & pmask(N);
  return P;
}

/* ------------------------------------------------------------------------ */
/* Operations                                                                */
/* ------------------------------------------------------------------------ */

uint32_t oracle_posit_neg(int N, uint32_t a) { return (0u - a) & pmask(N); }

uint32_t oracle_posit_add(int N, uint32_t a, uint32_t b) {
  pdec da = p_decode(N, a), db = p_decode(N, b);
  if (da.kind == P_NAR || db.kind == P_NAR) return p_nar(N);
  xnum xa = x_from_dec(&da), xb = x_from_dec(&db);
  xnum s = x_add(&xa, &xb);
  return x_round(N, &s);
}

uint32_t oracle_posit_sub(int N, uint32_t a, uint32_t b) {
  return oracle_posit_add(N, a, oracle_posit_neg(N, b));
}

uint32_t oracle_posit_mul(int N, uint32_t a, uint32_t b) {
  pdec da = p_decode(N, a), db = p_decode(N, b);
  if (da.kind == P_NAR || db.kind == P_NAR) return p_nar(N);
  if (da.kind == P_ZERO || db.kind == P_ZERO) return 0;
  xnum x;
  x_zero(&x);
  x.neg = da.neg ^ db.neg;
  unsigned __int128 prod = (unsigned __int128)p_sig(&da) * p_sig(&db);
  x_add_u128_at(&x, prod, p_lsbexp(&da) + p_lsbexp(&db) + XLSB);
  return x_round(N, &x);
}

uint32_t oracle_posit_div(int N, uint32_t a, uint32_t b) {
  pdec da = p_decode(N, a), db = p_decode(N, b);
  if (da.kind == P_NAR || db.kind == P_NAR || db.kind == P_ZERO) return p_nar(N);
  if (da.kind == P_ZERO) return 0;
  /* quotient with 64 extra bits; the remainder decides the sticky flag */
  unsigned __int128 num = (unsigned __int128)p_sig(&da) << 64;
  unsigned __int128 den = p_sig(&db);
  unsigned __int128 q = num / den, r = num % den;
  xnum x;
  x_zero(&x);
  x.neg = da.neg ^ db.neg;
  x_add_u128_at(&x, q, p_lsbexp(&da) - p_lsbexp(&db) - 64 + XLSB);
  x.sticky = r != 0;
  return x_round(N, &x);
}

/* floor(sqrt(v)), digit by digit */
static unsigned __int128 isqrt_u128(unsigned __int128 v) {
  unsigned __int128 r = 0, bit = (unsigned __int128)1 << 126;
  while (bit > v) bit >>= 2;
  while (bit) {
    if (v >= r + bit) {
      v -= r + bit;
      r = (r >> 1) + bit;
    } else {
      r >>= 1;
    }
    bit >>= 2;
  }
  return r;
}

uint32_t oracle_posit_sqrt(int N, uint32_t a) {
  pdec d = p_decode(N, a);
  if (d.kind == P_NAR || (d.kind == P_NORMAL && d.neg)) return p_nar(N);
  if (d.kind == P_ZERO) return 0;
  uint64_t s = p_sig(&d);
  int ex = p_lsbexp(&d);             /* |a| = s * 2^ex */
  if (ex & 1) { s <<= 1; ex -= 1; }  /* make the exponent even */
  unsigned __int128 v = (unsigned __int128)s << 80;
  unsigned __int128 r = isqrt_u128(v);
  assert(r * r <= v && (r + 1) * (r + 1) > v);
  xnum x;
  x_zero(&x);
  x_add_u128_at(&x, r, ex / 2 - 40 + XLSB);   /* sqrt(s*2^80) * 2^(ex/2-40) */
  x.sticky = r * r != v;
  return x_round(N, &x);
}

uint32_t oracle_posit_from_double(int N, double v) {
  if (isnan(v) || isinf(v)) return p_nar(N);
  if (v == 0.0) return 0;
  int ex;
  double m = frexp(fabs(v), &ex);                    /* |v| = m 2^ex     */
  uint64_t mant = (uint64_t)ldexp(m, 53);            /* exact integer    */
  int maxsc = p_maxscale(N);
  uint32_t P;
  if (ex - 1 >= maxsc) {
    P = p_maxpos(N);
  } else if (ex - 1 < -maxsc) {
    P = 1u;
  } else {
    xnum x;
    x_zero(&x);
    x.neg = v < 0;
    x_add_u128_at(&x, mant, ex - 53 + XLSB);
    return x_round(N, &x);
  }
  if (v < 0) P = (0u - P) & pmask(N);
  return P;
}

double oracle_posit_to_double(int N, uint32_t a) {
  pdec d = p_decode(N, a);
  if (d.kind == P_NAR) return NAN;
  if (d.kind == P_ZERO) return 0.0;
  double v = ldexp((double)p_sig(&d), p_lsbexp(&d));
  return d.neg ? -v : v;
}

int oracle_posit_fields(int N, uint32_t a, int* sign, int* k, int* e, int* fs,
                        uint32_t* f) {
  pdec d = p_decode(N, a);
  *sign = d.neg;
  *k = d.k;
  *e = d.e;
  *fs = d.fs;
  *f = d.f;
  return d.kind;
}

/* ------------------------------------------------------------------------ */
/* Array helpers                                                             */
/* ------------------------------------------------------------------------ */

void oracle_vec_from_double(int N, int64_t n, const double* x, uint32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = oracle_posit_from_double(N, x[i]);
}

void oracle_vec_to_double(int N, int64_t n, const uint32_t* p, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = oracle_posit_to_double(N, p[i]);
}

void oracle_vec_binop(int N, int op, int64_t n, const uint32_t* a,
                      const uint32_t* b, uint32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t r = 0;
    switch (op) {
      case 0: r = oracle_posit_add(N, a[i], b[i]); break;
      case 1: r = oracle_posit_sub(N, a[i], b[i]); break;
      case 2: r = oracle_posit_mul(N, a[i], b[i]); break;
      case 3: r = oracle_posit_div(N, a[i], b[i]); break;
      case 4: r = oracle_posit_sqrt(N, a[i]); break;
      default: abort();
    }
    out[i] = r;
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Rgemm (Section 3, Eq. (2))                                                */
/* ------------------------------------------------------------------------ */

static uint32_t p32_add(uint32_t a, uint32_t b) { return oracle_posit_add(32, a, b); }
static uint32_t p32_mul(uint32_t a, uint32_t b) { return oracle_posit_mul(32, a, b); }

static uint32_t gemm_one(int transa, int transb, int64_t i, int64_t j, int64_t k,
                         uint32_t alpha, const uint32_t* A, int64_t lda,
                         const uint32_t* B, int64_t ldb, uint32_t beta,
                         uint32_t cij) {
  if (alpha == 0 || k == 0) return beta == 0 ? 0u : p32_mul(beta, cij);
  uint32_t acc = 0;
  for (int64_t p = 0; p < k; ++p) {
    uint32_t a = transa ? A[p * lda + i] : A[i * lda + p];
    uint32_t b = transb ? B[j * ldb + p] : B[p * ldb + j];
    acc = p32_add(acc, p32_mul(a, b));
  }
  uint32_t r = p32_mul(alpha, acc);
  return beta == 0 ? r : p32_add(r, p32_mul(beta, cij));
}

void oracle_gemm(int transa, int transb, int64_t m, int64_t n, int64_t k,
                 uint32_t alpha, const uint32_t* A, int64_t lda,
                 const uint32_t* B, int64_t ldb, uint32_t beta, uint32_t* C,
                 int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      uint32_t cij = beta == 0 ? 0u : C[i * ldc + j];
      C[i * ldc + j] = gemm_one(transa, transb, i, j, k, alpha, A, lda, B,
                                ldb, beta, cij);
    }
}

void oracle_gemm_entries(int transa, int transb, int64_t k, uint32_t alpha,
                         const uint32_t* A, int64_t lda, const uint32_t* B,
                         int64_t ldb, uint32_t beta, int64_t count,
                         const int64_t* rows, const int64_t* cols,
                         const uint32_t* Cin, uint32_t* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < count; ++t)
    out[t] = gemm_one(transa, transb, rows[t], cols[t], k, alpha, A, lda, B,
                      ldb, beta, beta == 0 ? 0u : Cin[t]);
}
