// From the raw signed sum of a walk to the permanent, and the typed write of
// the result: shared by the single-matrix finishing kernel and the staged
// batch finish.
//
//   Glynn (Sec. 1.2 Eq. glynn, Eq. glynn_rectangle): E = 2^(n-1) (n-m)! per
//   (the e_m form is the case n = m: E = 2^(m-1) per);
//   square Ryser (Eq. ryser_square): E = (-1)^n per;
//   plain: E = per.
#pragma once
#include "device_common.h"
#include "internal.h"

namespace permgpu {

// the exponent of 2 in k!
__device__ inline int v2_factorial(int k) {
  int v = 0;
  for (int q = 2; q <= k; ++q) {
    int x = q;
    while ((x & 1) == 0) { ++v; x >>= 1; }
  }
  return v;
}

// a^-1 modulo 2^128 for odd a (Newton: each step doubles the correct bits)
__device__ inline u128 inverse_mod_2_128(u128 a) {
  u128 x = a;  // correct to 3 bits
  for (int i = 0; i < 6; ++i) x = x * ((u128)2 - a * x);
  return x;
}

// per from the integer sum E (kept modulo 2^128).  Glynn: E / (2^(n-1) (n-m)!)
// is exact as an integer; modulo 2^128 the division by 2^K (K = n-1 plus the
// power of two in (n-m)!) leaves per * odd modulo 2^(128-K), and the odd part
// of (n-m)! is inverted modulo 2^128; the result is sign-extended from bit
// 127-K.
__device__ inline i128 int_per(u128 E, int mode, int m, int n) {
  if (mode == FINISH_GLYNN) {
    const int k = n - m;
    const int v = v2_factorial(k);
    u128 odd = 1;
    for (int q = 2; q <= k; ++q) {
      int x = q;
      while ((x & 1) == 0) x >>= 1;
      odd *= (u128)x;
    }
    const int K = n - 1 + v;
    u128 y = K >= 128 ? 0 : (E >> K);             // (odd * per) mod 2^(128-K)
    y = y * inverse_mod_2_128(odd);               // per mod 2^(128-K)
    return K == 0 ? (i128)y : ((i128)(y << K)) >> K;
  }
  if (mode == FINISH_RYSER_SQ) return (n & 1) ? -(i128)E : (i128)E;
  return (i128)E;
}

// Floating-point normalisation of (rh, rl) [+ i (ih, il)] in double-double:
// Glynn scales by 2^-(n-1) and, for padding rows of 2^pad_e, 2^(-pad_e (n-m))
// (exact), then divides by (n-m)!; square Ryser takes the sign (-1)^n.
__device__ inline void fp_per(int mode, int m, int n, int pad_e, bool cplx, double &rh,
                              double &rl, double &ih, double &il) {
  if (mode == FINISH_GLYNN) {
    const double sc = __builtin_ldexp(1.0, -(n - 1) - pad_e * (n - m));
    rh *= sc; rl *= sc; ih *= sc; il *= sc;            // exact
    for (int q = 2; q <= n - m; ++q) {
      dd_div_d(rh, rl, (double)q);
      if (cplx) dd_div_d(ih, il, (double)q);
    }
  } else if (mode == FINISH_RYSER_SQ && (n & 1)) {
    rh = -rh; rl = -rl; ih = -ih; il = -il;
  }
}

// Write element i of an output array of type ot.
__device__ inline void write_fp(perm_out ot, double rh, double rl, double ih, double il, void *out,
                                size_t i) {
  double h1, l1, h2, l2;
  fast_two_sum(rh, rl, h1, l1);
  fast_two_sum(ih, il, h2, l2);
  double *o = (double *)out;
  switch (ot) {
    case PERM_OUT_F64: o[i] = h1; break;
    case PERM_OUT_DD: o[2 * i] = h1; o[2 * i + 1] = l1; break;
    case PERM_OUT_C128: o[2 * i] = h1; o[2 * i + 1] = h2; break;
    default: o[4 * i] = h1; o[4 * i + 1] = l1; o[4 * i + 2] = h2; o[4 * i + 3] = l2; break;
  }
}

__device__ inline void write_int(perm_out ot, i128 per, void *out, size_t i) {
  if (ot == PERM_OUT_I64) {
    ((int64_t *)out)[i] = (int64_t)per;
  } else {
    ((uint64_t *)out)[2 * i] = (uint64_t)(u128)per;
    ((uint64_t *)out)[2 * i + 1] = (uint64_t)((u128)per >> 64);
  }
}

}  // namespace permgpu
