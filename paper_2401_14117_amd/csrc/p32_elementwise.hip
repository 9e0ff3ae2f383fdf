// p32_elementwise.hip -- conversions and elementwise Posit(32,2) arithmetic
// (the paper's Add/Mul/Div/Sqrt kernels, Section 4.2): add, multiply and
// divide take the window-form fast path with the exact routines as fallback;
// the quotient and the square root come from binary64 estimates fixed up
// exactly with one fused multiply-add each.  Grid-stride loops; every element
// independent.
#include <hip/hip_runtime.h>
#include <math.h>

#include "p32_device.hpp"
#include "p32_launch.hpp"

namespace p32 {

__global__ void from_f64_kernel(int64_t n, const double* __restrict__ x, uint32_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    uint32_t r;
    if (!isfinite(v)) {
      r = kNaR;
    } else if (v == 0.0) {
      r = 0u;
    } else {
      const uint64_t bits = (uint64_t)__double_as_longlong(v);
      const bool neg = bits >> 63;
      const int bexp = (int)((bits >> 52) & 0x7FF);
      uint64_t mant = bits & ((((uint64_t)1) << 52) - 1);
      int x2;
      if (bexp == 0) {                 // subnormal: mant * 2^-1074
        x2 = -1074;
      } else {
        mant |= ((uint64_t)1) << 52;
        x2 = bexp - 1075;
      }
      r = round_general(neg, mant, x2, false);
    }
    out[i] = r;
  }
}

__global__ void to_f64_kernel(int64_t n, const uint32_t* __restrict__ p, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = p[i];
    double r;
    if (v == kNaR) {
      r = __longlong_as_double(0x7FF8000000000000LL);
    } else {
      const dec d = decode(v);
      r = d.s == 0 ? 0.0 : ldexp((double)d.s, d.sc - 27);
    }
    out[i] = r;
  }
}

// maxpos (big) or minpos with the given sign
__device__ __forceinline__ uint32_t saturated(bool neg, bool big) {
  const uint32_t p = big ? 0x7FFFFFFFu : 1u;
  return neg ? 0u - p : p;
}

// Sums and products that saturate are clamps, decided from the operands
// alone (a decoded value lies in [2^sc, 2^(sc+1))): a product at or beyond
// maxpos = 2^120 gives maxpos, one below minpos = 2^-120 gives minpos, and a
// sum of two same-signed values of which one is maxpos gives maxpos.
// Everything else takes the window-form fast path or the exact routines.
__global__ void elementwise_kernel(int op, int64_t n, const uint32_t* __restrict__ a,
                                   const uint32_t* __restrict__ b, uint32_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t x = a[i];
    const uint32_t y = op == 4 ? 0u : b[i];
    const bool xn = x == kNaR, yn = y == kNaR;
    uint32_t r;
    switch (op) {
      case 0:
      case 1: {
        const uint32_t yy = op == 1 ? 0u - y : y;
        if (xn || yn) {
          r = kNaR;
        } else {
          const bool same = x != 0u && yy != 0u && ((int32_t)x < 0) == ((int32_t)yy < 0);
          if (same && (x == 0x7FFFFFFFu || x == 0x80000001u || yy == 0x7FFFFFFFu || yy == 0x80000001u))
            r = saturated((int32_t)x < 0, true);
          else
            r = encode_win(add_win(win_of(x), win_of(yy)));
        }
        break;
      }
      case 2: {
        const dec dx = decode(x), dy = decode(y);
        const int s2 = dx.sc + dy.sc;
        if (xn || yn) r = kNaR;
        else if (dx.s == 0 || dy.s == 0) r = 0u;
        else if (s2 >= 120 || s2 <= -122) r = saturated((dx.s < 0) != (dy.s < 0), s2 >= 120);
        else r = encode_win(mul_win(dx, dy));
        break;
      }
      case 3: {
        const dec dx = decode(x), dy = decode(y);
        if (xn || yn || dy.s == 0) r = kNaR;         // x / 0 = NaR
        else r = encode_win(div_win(dx, dy, 1.0 / (double)(dy.s < 0 ? -(int64_t)dy.s : (int64_t)dy.s)));
        break;
      }
      default:
        r = p_sqrt(x);
        break;
    }
    out[i] = r;
  }
}

static dim3 grid_for(int64_t n) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  return dim3((unsigned)blocks);
}

int launch_from_f64(hipStream_t s, int64_t n, const double* x, uint32_t* out) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(from_f64_kernel, grid_for(n), dim3(256), 0, s, n, x, out);
  return launch_status();
}

int launch_to_f64(hipStream_t s, int64_t n, const uint32_t* p, double* out) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(to_f64_kernel, grid_for(n), dim3(256), 0, s, n, p, out);
  return launch_status();
}

int launch_elementwise(hipStream_t s, int op, int64_t n, const uint32_t* a, const uint32_t* b,
                       uint32_t* out) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(elementwise_kernel, grid_for(n), dim3(256), 0, s, op, n, a, b, out);
  return launch_status();
}

}  // namespace p32
