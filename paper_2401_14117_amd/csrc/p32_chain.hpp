// p32_chain.hpp -- one fused update rnd(c - rnd(l x)) with the Rgemm tile's
// k-step arithmetic, for the unblocked steps of the factorisations and the
// solves (the per-column rank-1 updates and substitutions that the blocked
// algorithms of Section 3 leave outside the Rgemm calls).  Every caller
// provides the rounding table (make_lut_entry) in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "p32_device.hpp"
#include "p32_gemm_tile.hpp"

namespace p32 {

// ---- one fused update of a running value -----------------------------------
// acc <- rnd(acc - rnd(m * x)) for one lane's running value acc (biased window
// form, as in the Rgemm tile), with the Rgemm's unchecked k-step arithmetic
// (staged operands, rounding parameters from the LDS table) when m, x and acc
// lie in its proven range: m and x nonzero with scales in [-53, 49], acc with
// scale in [-106, 100], so that the one step stays inside the table and the
// fast range.  Otherwise, and when the sum cancels or aligns past the fast
// path's reach, the lane takes the exact routines.  A zero m leaves acc as it
// is (acc - 0 is acc exactly).  dm: m decoded (not NaR); bx: x staged as an
// op(B) operand, nonzero and not NaR (a zero x leaves every running value
// unchanged and is skipped by the caller); x_ok: x's scale in the proven
// range.  Out of range, the table is indexed with stand-in operands (1 and
// -1), so every table access stays inside the table.
__device__ __forceinline__ bool scale_proven(int sc) { return (unsigned)(sc + 53) <= 102u; }

// the exact path of chain_update, out of line so that unrolled chains stay
// small in the instruction cache
static __device__ __noinline__ win chain_update_slow(win acc, dec dm, dec dx) {
  return bias(fms_win(unbias(acc), dm, dx));
}

__device__ __forceinline__ win chain_update(win acc, dec dm, int2 bx, bool x_ok, const lut_t* lut) {
  const bool m_ok = dm.s != 0 && scale_proven(dm.sc);
  const int2 a = m_ok ? stage_a(dm, true) : make_int2(-(1 << 30), 16 * 128);
  const int2 b = x_ok ? bx : make_int2(1 << 29, 0);
  uint32_t badbits = 0;
  const win pr = mul_unchecked(a, b, lut);
  win nacc = add_unchecked(acc, pr, lut, badbits);
  const bool acc_ok = (unsigned)(acc.e - EB + 106) <= 206u;   // a zero acc fails this
  if ((dm.s != 0) & (!(m_ok & x_ok & acc_ok) | (badbits > 63u))) {
    dec dx;
    dx.s = bx.x >> 2;
    dx.sc = bx.y >> 4;
    nacc = chain_update_slow(acc, dm, dx);
  }
  return dm.s != 0 ? nacc : acc;
}

// stand-in running value for lanes without a row (kept in the proven range)
__device__ __forceinline__ win idle_acc() {
  win w;
  w.h = 1 << 27;
  w.e = EB;
  return w;
}

// rnd(c - rnd(l x)) on patterns by chain_update: x given as its pattern xp
// (for the NaR test) and staged as an op(B) operand bx
__device__ __forceinline__ uint32_t fms_staged(uint32_t c, uint32_t l, uint32_t xp, int2 bx,
                                               const lut_t* lut) {
  if (c == kNaR || l == kNaR || xp == kNaR) return kNaR;
  if (bx.x == 0) return c;                        // c - rnd(l 0) = c
  return encode_win(unbias(chain_update(bias(win_of(c)), decode(l), bx, scale_proven(bx.y >> 4), lut)));
}

}  // namespace p32
