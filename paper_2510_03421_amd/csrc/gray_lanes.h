// Lane state of the Gray-code walks (engine and staged batches): the walk's
// vector v (column sums for Glynn, row sums for Ryser), the per-lane signed
// accumulation of the terms prod_j v_j, and the update / seed operations.
// Real kind: compensated (TwoSum) accumulation of plain 8-term partials, the
// last product multiply fused with the accumulation; complex kind: complex
// product chains, compensated real and imaginary sums; exact-integer kind:
// binary64 chunk products (exact below 2^52) multiplied modulo 2^128.
#pragma once
#include "device_common.h"
#include "internal.h"

namespace permgpu {
namespace walk {

// fuse the last product multiply with the accumulation (real kind)
#ifndef ENGINE_FUSED_ACC
#define ENGINE_FUSED_ACC 1
#endif
// product shape of the real kind: 0 = balanced tree, K > 0 = K interleaved
// chains (4 chains measured fastest at 4 waves per SIMD)
#ifndef ENGINE_PROD_CHAINS
#define ENGINE_PROD_CHAINS 4
#endif

// The update table lives in the constant address space: wave-uniform loads
// from it become scalar (SMEM) loads into SGPRs.
typedef __attribute__((address_space(4))) const double kdouble;

template <int NV, int KIND>
struct Lane;

// ---------------- real ----------------
template <int NV>
struct Lane<NV, ENGINE_REAL> {
  double v[NV];
  double s, hi, lo;
  __device__ __forceinline__ void zero_acc() { s = hi = lo = 0.0; }
  __device__ __forceinline__ void negate_acc() {
    s = -s;
    hi = -hi;
    lo = -lo;
  }
  __device__ __forceinline__ void load_base(const double *__restrict__ base) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = base[j];
  }
  // v += f * row, f in {0, 1} (per lane)
  __device__ __forceinline__ void seed_add(const double *__restrict__ row, double f) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = __builtin_fma(f, row[j], v[j]);
  }
  __device__ __forceinline__ void apply(const kdouble *__restrict__ row) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += row[j];
  }
  __device__ __forceinline__ double prod() const {
    if constexpr (ENGINE_PROD_CHAINS > 0)
      return prod_chains<NV, ENGINE_PROD_CHAINS>(v);
    else
      return prod_range<0, NV>(v);
  }
#if ENGINE_FUSED_ACC
  // s +- x*y with one rounding: the last multiply of the product and the
  // accumulation share an FMA
  __device__ __forceinline__ void split(double &x, double &y) const {
    if constexpr (ENGINE_PROD_CHAINS > 0)
      prod_split_chains<NV, ENGINE_PROD_CHAINS>(v, x, y);
    else
      prod_split_tree<NV>(v, x, y);
  }
  __device__ __forceinline__ void term_add() {
    double x, y;
    split(x, y);
    s = __builtin_fma(x, y, s);
  }
  __device__ __forceinline__ void term_sub() {
    double x, y;
    split(x, y);
    s = __builtin_fma(-x, y, s);
  }
#else
  __device__ __forceinline__ void term_add() { s += prod(); }
  __device__ __forceinline__ void term_sub() { s -= prod(); }
#endif
  __device__ __forceinline__ void flush() {
    dd_acc(hi, lo, s);
    s = 0.0;
  }
};

// ---------------- complex ----------------
template <int NV>
struct Lane<NV, ENGINE_CPLX> {
  double vr[NV], vi[NV];
  double sr, si, hr, lr, hi_, li;
  __device__ __forceinline__ void zero_acc() { sr = si = hr = lr = hi_ = li = 0.0; }
  __device__ __forceinline__ void negate_acc() {
    sr = -sr;
    si = -si;
    hr = -hr;
    lr = -lr;
    hi_ = -hi_;
    li = -li;
  }
  __device__ __forceinline__ void load_base(const double *__restrict__ base) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      vr[j] = base[2 * j];
      vi[j] = base[2 * j + 1];
    }
  }
  __device__ __forceinline__ void seed_add(const double *__restrict__ row, double f) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      vr[j] = __builtin_fma(f, row[2 * j], vr[j]);
      vi[j] = __builtin_fma(f, row[2 * j + 1], vi[j]);
    }
  }
  __device__ __forceinline__ void apply(const kdouble *__restrict__ row) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      vr[j] += row[2 * j];
      vi[j] += row[2 * j + 1];
    }
  }
  __device__ __forceinline__ void term_add() {
    double pr, pi;
    cprod_chains<NV, 4>(vr, vi, pr, pi);
    sr += pr;
    si += pi;
  }
  __device__ __forceinline__ void term_sub() {
    double pr, pi;
    cprod_chains<NV, 4>(vr, vi, pr, pi);
    sr -= pr;
    si -= pi;
  }
  __device__ __forceinline__ void flush() {
    dd_acc(hr, lr, sr);
    dd_acc(hi_, li, si);
    sr = si = 0.0;
  }
};

// ---------------- exact integer ----------------
template <int NV>
struct Lane<NV, ENGINE_INT> {
  double v[NV];
  u128 acc;
  int pl;       // product selector (int_chunk_count)
  bool nonneg;  // every factor >= 0 (0/1 Ryser): no sign
  __device__ __forceinline__ void zero_acc() { acc = 0; }
  __device__ __forceinline__ void negate_acc() { acc = (u128)0 - acc; }
  __device__ __forceinline__ void load_base(const double *__restrict__ base) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = base[j];
  }
  __device__ __forceinline__ void seed_add(const double *__restrict__ row, double f) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = __builtin_fma(f, row[j], v[j]);
  }
  __device__ __forceinline__ void apply(const kdouble *__restrict__ row) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += row[j];
  }
  __device__ __forceinline__ void term_add() { int_prod_acc<NV, false>(acc, v, pl, nonneg); }
  __device__ __forceinline__ void term_sub() { int_prod_acc<NV, true>(acc, v, pl, nonneg); }
  __device__ __forceinline__ void flush() {}
};

template <int KIND>
struct Comp {
  static constexpr int C = KIND == ENGINE_CPLX ? 2 : 1;
};

}  // namespace walk
}  // namespace permgpu
