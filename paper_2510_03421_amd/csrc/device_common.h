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

// ---- exact integer products (modulo 2^128) -------------------------------
// The factors are integer-valued doubles.  They are multiplied in binary64 in
// NCH chunks of K = ceil(NV / NCH) consecutive factors; the host picks NCH so
// that every chunk's product is below 2^52 in magnitude, so every partial
// product is exact.  A chunk's magnitude u < 2^52 becomes a 64-bit integer by
// adding 2^52 (the sum's significand then holds u exactly, and its exponent
// is fixed) and subtracting the bit pattern of 2^52 -- one floating-point add
// and one 32-bit subtract on the high word.  The magnitudes are multiplied
// modulo 2^128 in 32-bit limbs (the first pair exactly, 52 x 52 -> 104 bits;
// each further chunk with one row of limb products per 32-bit half of the
// chunk), and the chunks' signs, XORed, set the sign of the term.
// integral |x| < 2^53: split into high and low 32-bit parts exactly
__device__ __forceinline__ int64_t f64_to_i64_exact(double x) {
  double ax = __builtin_fabs(x);
  double h = __builtin_floor(ax * 0x1p-32);
  double l = __builtin_fma(-h, 0x1p32, ax);
  uint64_t u = ((uint64_t)(uint32_t)h << 32) | (uint64_t)(uint32_t)l;
  return x < 0 ? -(int64_t)u : (int64_t)u;
}
__device__ __forceinline__ uint64_t mag52(double x) {
  const double d = __builtin_fabs(x) + 0x1p52;
  return (uint64_t)__double_as_longlong(d) - (uint64_t)__double_as_longlong(0x1p52);
}
__device__ __forceinline__ uint32_t sign_word(double x) {
  return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32);  // bit 31 = sign
}

// a, b < 2^52: the exact product (< 2^104) as (lo, hi)
__device__ __forceinline__ void mul52x52(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t x = (uint64_t)a0 * b0;
  uint64_t y = (uint64_t)a0 * b1 + (x >> 32);
  y = (uint64_t)a1 * b0 + y;                      // < 2^53 + 2^32
  const uint64_t z = (uint64_t)a1 * b1 + (y >> 32);
  lo = (x & 0xffffffffull) | (y << 32);
  hi = z;
}

// (lo, hi) <- (lo, hi) * c modulo 2^128, c < 2^52
__device__ __forceinline__ void mul128x52(uint64_t &lo, uint64_t &hi, uint64_t c) {
  const uint32_t p0 = (uint32_t)lo, p1 = (uint32_t)(lo >> 32);
  const uint32_t p2 = (uint32_t)hi, p3 = (uint32_t)(hi >> 32);
  const uint32_t c0 = (uint32_t)c, c1 = (uint32_t)(c >> 32);
  const uint64_t u0 = (uint64_t)p0 * c0;
  const uint64_t u1 = (uint64_t)p1 * c0 + (u0 >> 32);
  const uint64_t u2 = (uint64_t)p2 * c0 + (u1 >> 32);
  const uint32_t u3 = p3 * c0 + (uint32_t)(u2 >> 32);
  const uint64_t w1 = (uint64_t)p0 * c1 + (uint32_t)u1;
  const uint64_t w2 = (uint64_t)p1 * c1 + (uint32_t)u2 + (w1 >> 32);
  const uint32_t w3 = p2 * c1 + u3 + (uint32_t)(w2 >> 32);
  lo = (u0 & 0xffffffffull) | (w1 << 32);
  hi = (w2 & 0xffffffffull) | ((uint64_t)w3 << 32);
}

// chunk C (factors [C K, min((C+1) K, NV))) of NCH: multiply its magnitude
// into (lo, hi) and its sign into sg
template <int NV, int NCH, int C, class T>
__device__ __forceinline__ void int_chunks(const T &v, uint64_t &lo, uint64_t &hi, uint32_t &sg) {
  constexpr int K = (NV + NCH - 1) / NCH;
  constexpr int L = C * K, R = (C + 1) * K < NV ? (C + 1) * K : NV;
  if constexpr (L < NV) {
    const double x = prod_range<L, R>(v);
    const uint64_t u = mag52(x);
    if constexpr (C == 0) {
      lo = u;
      hi = 0;
      sg = sign_word(x);
    } else {
      if constexpr (C == 1) mul52x52(lo, u, lo, hi);
      else mul128x52(lo, hi, u);
      sg ^= sign_word(x);
    }
    int_chunks<NV, NCH, C + 1>(v, lo, hi, sg);
  }
}

// The chunk counts the term code is instantiated for (index = the host's
// product selector): with K = ceil(NV / NCH) factors per chunk.
__host__ __device__ constexpr int int_chunk_count(int sel, int nv) {
  return sel == 0 ? nv : sel == 1 ? 8 : sel == 2 ? 6 : sel == 3 ? 4 : sel == 4 ? 3 : sel == 5 ? 2 : 1;
}
constexpr int kIntProdSelectors = 7;

template <int NV, int NCH, class T>
__device__ __forceinline__ void int_prod_nch(const T &v, uint64_t &lo, uint64_t &hi, uint32_t &sg) {
  constexpr int N = NCH < NV ? NCH : NV;
  int_chunks<NV, N, 0>(v, lo, hi, sg);
}

// acc += (-1)^NEG prod_j v_j modulo 2^128; sel picks the chunk count (uniform)
// and nonneg skips the sign when every factor is known to be >= 0.
template <int NV, bool NEG, class T>
__device__ __forceinline__ void int_prod_acc(u128 &acc, const T &v, int sel, bool nonneg) {
  uint64_t lo = 0, hi = 0;
  uint32_t sg = 0;
  switch (sel) {
    case 0: int_prod_nch<NV, NV>(v, lo, hi, sg); break;
    case 1: int_prod_nch<NV, 8>(v, lo, hi, sg); break;
    case 2: int_prod_nch<NV, 6>(v, lo, hi, sg); break;
    case 3: int_prod_nch<NV, 4>(v, lo, hi, sg); break;
    case 4: int_prod_nch<NV, 3>(v, lo, hi, sg); break;
    case 5: int_prod_nch<NV, 2>(v, lo, hi, sg); break;
    default: int_prod_nch<NV, 1>(v, lo, hi, sg); break;
  }
  u128 m = ((u128)hi << 64) | lo;
  if (!nonneg) {
    // negative product: two's complement negation, (m ^ mask) - mask
    const u128 mask = (u128)(i128)((int32_t)sg >> 31);
    m = (m ^ mask) - mask;
  }
  if constexpr (NEG) acc -= m;
  else acc += m;
}

// ---- wave-level shuffles of 64-bit and 128-bit values ----
__device__ __forceinline__ double shfl_xor_d(double x, int m, int width) {
  return __shfl_xor(x, m, width);
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m, int width) {
  return (uint64_t)__shfl_xor((unsigned long long)x, m, width);
}

}  // namespace permgpu
