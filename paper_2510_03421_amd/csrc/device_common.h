// Device-side helpers shared by the kernels: error-free transformations,
// double-double accumulation, product trees and 128-bit integer arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace permgpu {

typedef unsigned __int128 u128;
typedef __int128 i128;

// ---- error-free transformations (Knuth TwoSum, Dekker Fast2Sum, FMA TwoProd)
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}
// (hi, lo) += (bhi, blo), normalised double-double addition
__device__ __forceinline__ void dd_add(double &hi, double &lo, double bhi, double blo) {
  double s, e, t, f;
  two_sum(hi, bhi, s, e);
  two_sum(lo, blo, t, f);
  e += t;
  fast_two_sum(s, e, s, e);
  e += f;
  fast_two_sum(s, e, hi, lo);
}
// running compensated sum: hi carries the sum, lo collects the rounding errors
__device__ __forceinline__ void dd_acc(double &hi, double &lo, double x) {
  double s, e;
  two_sum(hi, x, s, e);
  hi = s;
  lo += e;
}
__device__ __forceinline__ void dd_mul_d(double &hi, double &lo, double b) {
  double p = hi * b;
  double e = __builtin_fma(hi, b, -p);
  e = __builtin_fma(lo, b, e);
  fast_two_sum(p, e, hi, lo);
}
// (hi, lo) / d for a double d: one correction step of the quotient
__device__ __forceinline__ void dd_div_d(double &hi, double &lo, double d) {
  double q1 = hi / d;
  double p = q1 * d;
  double pe = __builtin_fma(q1, d, -p);
  double r = ((hi - p) - pe) + lo;
  double q2 = r / d;
  fast_two_sum(q1, q2, hi, lo);
}

// ---- product trees over a register array (balanced halving) ----
template <int L, int R, class T>
__device__ __forceinline__ double prod_range(const T &v) {
  if constexpr (R - L == 1) {
    return v[L];
  } else {
    constexpr int M = L + (R - L) / 2;
    return prod_range<L, M>(v) * prod_range<M, R>(v);
  }
}

// product of v[0..NV) as K interleaved left-to-right chains combined at the
// end: fewer live temporaries than the balanced tree (K instead of NV/2)
template <int NV, int K, class T>
__device__ __forceinline__ double prod_chains(const T &v) {
  if constexpr (NV < 2 * K) {
    return prod_range<0, NV>(v);
  } else {
    double c[K];
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = v[k];
#pragma unroll
    for (int j = K; j < NV; ++j) c[j % K] *= v[j];
    return prod_range<0, K>(c);
  }
}

// The same products split into two final factors (x, y) with x*y the full
// product, so that an accumulation s +- x*y can be one FMA.
template <int NV, class T>
__device__ __forceinline__ void prod_split_tree(const T &v, double &x, double &y) {
  if constexpr (NV == 1) {
    x = v[0];
    y = 1.0;
  } else {
    constexpr int M = NV / 2;
    x = prod_range<0, M>(v);
    y = prod_range<M, NV>(v);
  }
}
template <int NV, int K, class T>
__device__ __forceinline__ void prod_split_chains(const T &v, double &x, double &y) {
  if constexpr (NV < 2 * K || K < 2) {
    prod_split_tree<NV>(v, x, y);
  } else {
    double c[K];
#pragma unroll
    for (int k = 0; k < K; ++k) c[k] = v[k];
#pragma unroll
    for (int j = K; j < NV; ++j) c[j % K] *= v[j];
    x = prod_range<0, K / 2>(c);
    y = prod_range<K / 2, K>(c);
  }
}

// complex product over (vr, vi) with explicit FMA:
//   (a + ib)(c + id) = (ac - bd) + i(ad + bc)
__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double &cr,
                                     double &ci) {
  double t = ai * bi;
  double u = ai * br;
  cr = __builtin_fma(ar, br, -t);
  ci = __builtin_fma(ar, bi, u);
}
template <int L, int R, class T>
__device__ __forceinline__ void cprod_range(const T &vr, const T &vi, double &pr, double &pi) {
  if constexpr (R - L == 1) {
    pr = vr[L];
    pi = vi[L];
  } else {
    constexpr int M = L + (R - L) / 2;
    double ar, ai, br, bi;
    cprod_range<L, M>(vr, vi, ar, ai);
    cprod_range<M, R>(vr, vi, br, bi);
    cmul(ar, ai, br, bi, pr, pi);
  }
}

// complex product as K interleaved chains of complex multiplies, combined by
// a balanced tree at the end
template <int NV, int K, class T>
__device__ __forceinline__ void cprod_chains(const T &vr, const T &vi, double &pr, double &pi) {
  if constexpr (NV < 2 * K) {
    cprod_range<0, NV>(vr, vi, pr, pi);
  } else {
    double cr[K], ci[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      cr[k] = vr[k];
      ci[k] = vi[k];
    }
#pragma unroll
    for (int j = K; j < NV; ++j) {
      double r, i;
      cmul(cr[j % K], ci[j % K], vr[j], vi[j], r, i);
      cr[j % K] = r;
      ci[j % K] = i;
    }
    cprod_range<0, K>(cr, ci, pr, pi);
  }
}

// ---- exact integer products: binary64 chunks of 2^PL factors (exact because
// the host guarantees every chunk's bound is below 2^53), then mod 2^128.
__device__ __forceinline__ int64_t f64_to_i64_exact(double x) {
  // |x| < 2^53 and integral: split into high and low 32-bit parts exactly
  double ax = __builtin_fabs(x);
  double h = __builtin_floor(ax * 0x1p-32);
  double l = __builtin_fma(-h, 0x1p32, ax);
  uint64_t u = ((uint64_t)(uint32_t)h << 32) | (uint64_t)(uint32_t)l;
  return x < 0 ? -(int64_t)u : (int64_t)u;
}
template <int NV, int C, int C0, class T>
__device__ __forceinline__ void int_chunks(const T &v, u128 &acc) {
  if constexpr (C0 < NV) {
    constexpr int C1 = (C0 + C < NV) ? C0 + C : NV;
    const double x = prod_range<C0, C1>(v);
    const u128 xi = (u128)(i128)f64_to_i64_exact(x);
    if constexpr (C0 == 0)
      acc = xi;
    else
      acc = acc * xi;
    int_chunks<NV, C, C1>(v, acc);
  }
}
template <int NV, class T>
__device__ __forceinline__ u128 int_prod(const T &v, int pl) {
  u128 acc = 0;
  switch (pl) {
    case 0: int_chunks<NV, 1, 0>(v, acc); break;
    case 1: int_chunks<NV, 2, 0>(v, acc); break;
    case 2: int_chunks<NV, 4, 0>(v, acc); break;
    default: int_chunks<NV, 8, 0>(v, acc); break;
  }
  return acc;
}

// ---- wave-level shuffles of 64-bit and 128-bit values ----
__device__ __forceinline__ double shfl_xor_d(double x, int m, int width) {
  return __shfl_xor(x, m, width);
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m, int width) {
  return (uint64_t)__shfl_xor((unsigned long long)x, m, width);
}

}  // namespace permgpu
