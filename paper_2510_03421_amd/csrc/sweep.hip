// The column-sweep form of the definition (Sec. 1.1 Eq.
// rectangular_permanent_definition): for an m x n matrix (m <= n), let g_j[R]
// be the sum over injective maps of the rows R (a subset of the m rows) into
// columns 0..j of the products of their entries.  Then g_{-1}[{}] = 1 and
//
//   g_j[R] = g_{j-1}[R] + sum_{i in R} a_ij g_{j-1}[R \ {i}]
//
// (column j is either unused or taken by one row i of R), and per(A) =
// g_{n-1}[all m rows].  The sum regroups the definition's products without
// any subtraction of computed values: the floating-point result is off by at
// most about (m + n) u per(|A|), however the inclusion-exclusion forms cancel.
//
// GPU layout: the 2^m states of one column in a flat array indexed by the
// row bitmask, two buffers used in turn.  One thread per state R; column j
// only needs the states whose size k can still reach m and is reachable,
// max(0, m - (n - j)) <= k <= min(j + 1, m); the others are not touched (the
// states read at column j + 1 were all written at column j).  Exact integers
// are kept modulo 2^128.
#include "device_common.h"
#include "finish_common.h"
#include "internal.h"

namespace permgpu {
namespace {

__device__ __forceinline__ void rd(perm_dtype dt, const void *dA, int64_t lda, int tr, int i,
                                   int j, double &re, double &im) {
  const int64_t o = tr ? (int64_t)j * lda + i : (int64_t)i * lda + j;
  im = 0.0;
  switch (dt) {
    case PERM_F64: re = ((const double *)dA)[o]; break;
    case PERM_C128:
      re = ((const double *)dA)[2 * o];
      im = ((const double *)dA)[2 * o + 1];
      break;
    case PERM_I64: re = 0.0; break;  // integer input is read as int64 below
    default: re = ((const uint8_t *)dA)[o] ? 1.0 : 0.0; break;
  }
}
__device__ __forceinline__ int64_t rdi(perm_dtype dt, const void *dA, int64_t lda, int tr, int i,
                                       int j) {
  const int64_t o = tr ? (int64_t)j * lda + i : (int64_t)i * lda + j;
  return dt == PERM_I64 ? ((const int64_t *)dA)[o] : (((const uint8_t *)dA)[o] ? 1 : 0);
}

// one column of the sweep: states R with lo <= |R| <= hi
template <int KIND>
__global__ __launch_bounds__(256) void sweep_kernel(int m, int j, int lo, int hi, perm_dtype dt,
                                                    const void *dA, int64_t lda, int tr,
                                                    const void *oldv, void *newv) {
  const uint64_t R = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >> m) return;
  const int k = __builtin_popcountll(R);
  if (k < lo || k > hi) return;
  if constexpr (KIND == ENGINE_INT) {
    const uint64_t *o = (const uint64_t *)oldv;
    u128 acc = ((u128)o[2 * R + 1] << 64) | o[2 * R];
    for (uint64_t r = R; r; r &= r - 1) {
      const int i = __builtin_ctzll(r);
      const int64_t a = rdi(dt, dA, lda, tr, i, j);
      if (a == 0) continue;
      const uint64_t S = R ^ (1ull << i);
      const u128 x = ((u128)o[2 * S + 1] << 64) | o[2 * S];
      acc += x * (u128)(i128)a;
    }
    uint64_t *w = (uint64_t *)newv;
    w[2 * R] = (uint64_t)acc;
    w[2 * R + 1] = (uint64_t)(acc >> 64);
  } else if constexpr (KIND == ENGINE_CPLX) {
    const double *o = (const double *)oldv;
    double ar = o[2 * R], ai = o[2 * R + 1];
    for (uint64_t r = R; r; r &= r - 1) {
      const int i = __builtin_ctzll(r);
      double xr, xi;
      rd(dt, dA, lda, tr, i, j, xr, xi);
      const uint64_t S = R ^ (1ull << i);
      const double br = o[2 * S], bi = o[2 * S + 1];
      ar = __builtin_fma(xr, br, __builtin_fma(-xi, bi, ar));
      ai = __builtin_fma(xr, bi, __builtin_fma(xi, br, ai));
    }
    double *w = (double *)newv;
    w[2 * R] = ar;
    w[2 * R + 1] = ai;
  } else {
    const double *o = (const double *)oldv;
    double acc = o[R];
    for (uint64_t r = R; r; r &= r - 1) {
      const int i = __builtin_ctzll(r);
      double x, xi;
      if (dt == PERM_I64) x = (double)rdi(dt, dA, lda, tr, i, j);
      else rd(dt, dA, lda, tr, i, j, x, xi);
      acc = __builtin_fma(x, o[R ^ (1ull << i)], acc);
    }
    ((double *)newv)[R] = acc;
  }
}

// g_{-1}: 1 at the empty set (the buffers start zeroed)
__global__ void sweep_init_kernel(int kind, void *v) {
  if (kind == ENGINE_INT) {
    ((uint64_t *)v)[0] = 1;
  } else {
    ((double *)v)[0] = 1.0;
  }
}

// the value at the full set, written in the output type
__global__ void sweep_finish_kernel(int kind, int m, const void *v, perm_out ot, void *out) {
  const uint64_t F = (1ull << m) - 1;
  if (kind == ENGINE_INT) {
    const uint64_t *p = (const uint64_t *)v;
    write_int(ot, (i128)(((u128)p[2 * F + 1] << 64) | p[2 * F]), out, 0);
  } else if (kind == ENGINE_CPLX) {
    const double *p = (const double *)v;
    write_fp(ot, p[2 * F], 0.0, p[2 * F + 1], 0.0, out, 0);
  } else {
    write_fp(ot, ((const double *)v)[F], 0.0, 0.0, 0.0, out, 0);
  }
}

}  // namespace

hipError_t launch_sweep(int kind, int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                        void *buf0, void *buf1, size_t state_bytes, perm_out ot, void *dOut,
                        hipStream_t s, int ncols) {
  const size_t bytes = state_bytes << m;
  hipError_t e = hipMemsetAsync(buf0, 0, bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(buf1, 0, bytes, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sweep_init_kernel, dim3(1), dim3(1), 0, s, kind, buf0);
  e = hipGetLastError();
  void *cur = buf0, *nxt = buf1;
  const uint64_t states = 1ull << m;
  const unsigned grid = (unsigned)((states + 255) / 256);
  for (int j = 0; j < ncols && e == hipSuccess; ++j) {
    // sizes that can still reach m with the n - 1 - j columns left
    const int lo = m - (n - 1 - j) > 0 ? m - (n - 1 - j) : 0;
    const int hi = j + 1 < m ? j + 1 : m;
    switch (kind) {
      case ENGINE_INT:
        hipLaunchKernelGGL(sweep_kernel<ENGINE_INT>, dim3(grid), dim3(256), 0, s, m, j, lo, hi, dt,
                           dA, lda, tr, cur, nxt);
        break;
      case ENGINE_CPLX:
        hipLaunchKernelGGL(sweep_kernel<ENGINE_CPLX>, dim3(grid), dim3(256), 0, s, m, j, lo, hi,
                           dt, dA, lda, tr, cur, nxt);
        break;
      default:
        hipLaunchKernelGGL(sweep_kernel<ENGINE_REAL>, dim3(grid), dim3(256), 0, s, m, j, lo, hi,
                           dt, dA, lda, tr, cur, nxt);
        break;
    }
    e = hipGetLastError();
    void *t = cur;
    cur = nxt;
    nxt = t;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sweep_finish_kernel, dim3(1), dim3(1), 0, s, kind, m, cur, ot, dOut);
  return hipGetLastError();
}

}  // namespace permgpu
