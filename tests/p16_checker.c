/*
 * Exhaustive check of the oracle's Posit(16,2) add, mul and div over all
 * 2^32 operand pairs, and sqrt over all 2^16 operands (test code).
 *
 * Independent of the oracle: values are decoded with count-leading-bits
 * arithmetic into doubles (every Posit(16,2) and Posit(17,2) value is exact in
 * FP64), and results are rounded by binary search for the neighbours u <= x < w
 * followed by a comparison with the 17-bit midpoint pattern 2U+1 (ties to the
 * even pattern).  Comparisons with the exact target are exact: products and
 * quotient cross-products fit in 53 bits, sums are compared in 128-bit fixed
 * point with unit 2^-60 (the spacing of the finest 17-bit posit).
 *
 * Usage: p16_checker [stride]  -- checks every stride-th first operand.
 * Prints the number of mismatches; exit status 0 when there are none.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/posit_oracle.h"

static double v16[1 << 16];
static double v17[1 << 17];

static double decode_clz(int N, uint32_t p) {
  uint32_t msk = (1u << N) - 1u;
  p &= msk;
  if (p == 0) return 0.0;
  if (p == (1u << (N - 1))) return NAN;
  int neg = (p >> (N - 1)) & 1u;
  if (neg) p = (0u - p) & msk;
  uint32_t x = p << (33 - N);            /* body left-aligned at bit 31 */
  int lead = (int)(x >> 31);
  int run;                               /* regime run length */
  if (lead) run = (~x) ? __builtin_clz(~x) : 32;
  else run = x ? __builtin_clz(x) : 32;
  if (run > N - 1) run = N - 1;
  int k = lead ? run - 1 : -run;
  int remaining = N - 1 - run - 1;       /* bits after the terminator */
  if (remaining < 0) remaining = 0;
  uint32_t rest = (run + 1 < 32) ? (x << (run + 1)) : 0u;
  int e = (int)(rest >> 30);             /* missing bits shift in as 0 */
  int fb = remaining - 2 > 0 ? remaining - 2 : 0;
  uint32_t f = fb ? (rest << 2) >> (32 - fb) : 0u;
  double v = ldexp(1.0 + ldexp((double)f, -fb), 4 * k + e);
  return neg ? -v : v;
}

typedef __int128 i128;
static i128 fx(double v) { return (i128)ldexp(v, 60); }

/* cmp(v) = sign(v - target) for positive targets */
typedef int (*cmpfn)(double v, const void* ctx);

static uint32_t round_pos(cmpfn cmp, const void* ctx) {
  const uint32_t maxpos = 0x7FFF;
  if (cmp(v16[maxpos], ctx) <= 0) return maxpos;
  if (cmp(v16[1], ctx) >= 0) return 1;
  uint32_t lo = 1, hi = maxpos;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) / 2;
    if (cmp(v16[mid], ctx) <= 0) lo = mid; else hi = mid;
  }
  if (cmp(v16[lo], ctx) == 0) return lo;
  int c = cmp(v17[2 * lo + 1], ctx);
  if (c > 0) return lo;
  if (c < 0) return lo + 1;
  return (lo & 1u) ? lo + 1 : lo;
}

typedef struct { double a, b; } pair;
static int cmp_mul(double v, const void* c) {
  const pair* p = c;
  double x = fabs(p->a * p->b);
  return (v > x) - (v < x);
}
static int cmp_div(double v, const void* c) {
  const pair* p = c;
  double l = v * fabs(p->b), r = fabs(p->a);
  return (l > r) - (l < r);
}
typedef struct { i128 s; } sumc;
static int cmp_add(double v, const void* c) {
  const sumc* p = c;
  i128 fv = fx(v);
  return (fv > p->s) - (fv < p->s);
}
static int cmp_sqrt(double v, const void* c) {
  double a = *(const double*)c, l = v * v;
  return (l > a) - (l < a);
}

static uint32_t signed_result(uint32_t P, int neg) { return neg ? ((0u - P) & 0xFFFFu) : P; }

static uint32_t chk_add(uint32_t a, uint32_t b) {
  double va = v16[a], vb = v16[b];
  if (isnan(va) || isnan(vb)) return 0x8000;
  i128 s = fx(va) + fx(vb);
  if (s == 0) return 0;
  sumc c = {s < 0 ? -s : s};
  return signed_result(round_pos(cmp_add, &c), s < 0);
}
static uint32_t chk_mul(uint32_t a, uint32_t b) {
  double va = v16[a], vb = v16[b];
  if (isnan(va) || isnan(vb)) return 0x8000;
  if (va == 0 || vb == 0) return 0;
  pair c = {va, vb};
  return signed_result(round_pos(cmp_mul, &c), (va < 0) != (vb < 0));
}
static uint32_t chk_div(uint32_t a, uint32_t b) {
  double va = v16[a], vb = v16[b];
  if (isnan(va) || isnan(vb) || vb == 0) return 0x8000;
  if (va == 0) return 0;
  pair c = {va, vb};
  return signed_result(round_pos(cmp_div, &c), (va < 0) != (vb < 0));
}
static uint32_t chk_sqrt(uint32_t a) {
  double va = v16[a];
  if (isnan(va) || va < 0) return 0x8000;
  if (va == 0) return 0;
  return round_pos(cmp_sqrt, &va);
}

int main(int argc, char** argv) {
  int stride = argc > 1 ? atoi(argv[1]) : 1;
  for (uint32_t p = 0; p < (1u << 16); ++p) v16[p] = decode_clz(16, p);
  for (uint32_t p = 0; p < (1u << 17); ++p) v17[p] = decode_clz(17, p);
  for (uint32_t p = 1; p < 0x7FFF; ++p)
    if (!(v16[p] < v16[p + 1])) { printf("decode not monotone at %u\n", p); return 2; }
  long long bad = 0, checked = 0;
  for (uint32_t a = 0; a < (1u << 16); ++a) {
    uint32_t s = oracle_posit_sqrt(16, a);
    if (s != chk_sqrt(a)) { if (bad < 10) printf("sqrt %04x\n", a); ++bad; }
  }
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad, checked)
  for (int ai = 0; ai < (1 << 16); ai += stride) {
    uint32_t a = (uint32_t)ai;
    for (uint32_t b = 0; b < (1u << 16); ++b) {
      uint32_t r1 = oracle_posit_add(16, a, b), r2 = oracle_posit_mul(16, a, b),
               r3 = oracle_posit_div(16, a, b);
      int m = (r1 != chk_add(a, b)) + (r2 != chk_mul(a, b)) + (r3 != chk_div(a, b));
      if (m) {
#pragma omp critical
        if (bad < 10) printf("mismatch a=%04x b=%04x\n", a, b);
        bad += m;
      }
      checked += 3;
    }
  }
  printf("checked %lld results, %lld mismatches\n", checked, bad);
  return bad != 0;
}
