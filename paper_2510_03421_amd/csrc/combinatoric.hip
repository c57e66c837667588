// The definition on the GPU (Sec. 1.1 Eq. rectangular_permanent_definition;
// cost m n!/(n-m)!, Sec. 1.2): one product per injective map s:[m]->[n].
//
// Maps are ranked in lexicographic order of (s(0), ..., s(m-1)): the rank's
// mixed-radix digits d_i in bases n, n-1, ..., n-m+1 pick s(i) as the d_i-th
// column not used by rows 0..i-1.  Each thread takes a contiguous range of
// ranks; A is staged in LDS.  Real products are summed with a compensated
// accumulator, integer products modulo 2^128.
#include "device_common.h"
#include "internal.h"

namespace permgpu {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int nth_unused(uint64_t used, int d) {
  // index of the d-th zero bit of `used` (0-based)
  int j = 0;
  for (;; ++j) {
    if (!((used >> j) & 1u)) {
      if (d == 0) return j;
      --d;
    }
  }
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void combinatoric_kernel(int m, int n, perm_dtype dt,
                                                                const void *dA, int64_t lda,
                                                                int tr, uint64_t total,
                                                                void *partials) {
  extern __shared__ double sa[];  // m*n (x2 for complex) entries
  constexpr int C = KIND == ENGINE_CPLX ? 2 : 1;
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const int64_t o = tr ? (int64_t)j * lda + i : (int64_t)i * lda + j;
    double re = 0.0, im = 0.0;
    switch (dt) {
      case PERM_F64: re = ((const double *)dA)[o]; break;
      case PERM_C128:
        re = ((const double *)dA)[2 * o];
        im = ((const double *)dA)[2 * o + 1];
        break;
      case PERM_I64: {
        // the integer kernel keeps the raw 64-bit value in the slot
        const int64_t v = ((const int64_t *)dA)[o];
        re = KIND == ENGINE_INT ? __longlong_as_double(v) : (double)v;
        break;
      }
      default: {
        const int v = ((const uint8_t *)dA)[o] ? 1 : 0;
        re = KIND == ENGINE_INT ? __longlong_as_double((int64_t)v) : (double)v;
        break;
      }
    }
    sa[e * C] = re;
    if (C == 2) sa[e * C + 1] = im;
  }
  __syncthreads();
  const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t r0 = (uint64_t)(((u128)total * t) / T);
  const uint64_t r1 = (uint64_t)(((u128)total * (t + 1)) / T);
  double hi = 0.0, lo = 0.0, hi2 = 0.0, lo2 = 0.0;
  u128 acc = 0;
  for (uint64_t r = r0; r < r1; ++r) {
    // digits, least significant (last row) first
    int dig[64];
    uint64_t x = r;
    for (int i = m - 1; i >= 0; --i) {
      const uint64_t base = (uint64_t)(n - i);
      dig[i] = (int)(x % base);
      x /= base;
    }
    uint64_t used = 0;
    if constexpr (KIND == ENGINE_REAL) {
      double p = 1.0;
      for (int i = 0; i < m; ++i) {
        const int j = nth_unused(used, dig[i]);
        used |= 1ull << j;
        p = i == 0 ? sa[i * n + j] : p * sa[i * n + j];
      }
      dd_acc(hi, lo, p);
    } else if constexpr (KIND == ENGINE_CPLX) {
      double pr = 1.0, pi = 0.0;
      for (int i = 0; i < m; ++i) {
        const int j = nth_unused(used, dig[i]);
        used |= 1ull << j;
        const double ar = sa[2 * (i * n + j)], ai = sa[2 * (i * n + j) + 1];
        if (i == 0) {
          pr = ar;
          pi = ai;
        } else {
          const double qr = pr * ar - pi * ai;
          const double qi = pr * ai + pi * ar;
          pr = qr;
          pi = qi;
        }
      }
      dd_acc(hi, lo, pr);
      dd_acc(hi2, lo2, pi);
    } else {
      u128 p = 1;
      for (int i = 0; i < m; ++i) {
        const int j = nth_unused(used, dig[i]);
        used |= 1ull << j;
        const int64_t v = __double_as_longlong(sa[i * n + j]);
        p *= (u128)(i128)v;
      }
      acc += p;
    }
  }
  // workgroup reduction -> one partial
  __shared__ double red[kThreads / 64][4];
  __shared__ uint64_t ired[kThreads / 64][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if constexpr (KIND == ENGINE_INT) {
    uint64_t l64 = (uint64_t)acc, h64 = (uint64_t)(acc >> 64);
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t ol = shfl_xor_u64(l64, off, 64), oh = shfl_xor_u64(h64, off, 64);
      const u128 y = (((u128)h64) << 64 | l64) + (((u128)oh) << 64 | ol);
      l64 = (uint64_t)y;
      h64 = (uint64_t)(y >> 64);
    }
    if (lane == 0) { ired[wave][0] = l64; ired[wave][1] = h64; }
    __syncthreads();
    if (threadIdx.x == 0) {
      u128 y = 0;
      for (int w = 0; w < kThreads / 64; ++w) y += ((u128)ired[w][1]) << 64 | ired[w][0];
      ((uint64_t *)partials)[2 * blockIdx.x] = (uint64_t)y;
      ((uint64_t *)partials)[2 * blockIdx.x + 1] = (uint64_t)(y >> 64);
    }
  } else {
    double a, b, c = 0.0, d = 0.0;
    fast_two_sum(hi, lo, a, b);
    if (C == 2) fast_two_sum(hi2, lo2, c, d);
    for (int off = 32; off > 0; off >>= 1) {
      double oa = shfl_xor_d(a, off, 64), ob = shfl_xor_d(b, off, 64);
      dd_add(a, b, oa, ob);
      if (C == 2) {
        double oc = shfl_xor_d(c, off, 64), od = shfl_xor_d(d, off, 64);
        dd_add(c, d, oc, od);
      }
    }
    if (lane == 0) { red[wave][0] = a; red[wave][1] = b; red[wave][2] = c; red[wave][3] = d; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double A = red[0][0], B = red[0][1], Cc = red[0][2], D = red[0][3];
      for (int w = 1; w < kThreads / 64; ++w) {
        dd_add(A, B, red[w][0], red[w][1]);
        dd_add(Cc, D, red[w][2], red[w][3]);
      }
      double *p = (double *)partials + 2 * C * blockIdx.x;
      p[0] = A;
      p[1] = B;
      if (C == 2) { p[2] = Cc; p[3] = D; }
    }
  }
}

}  // namespace

hipError_t launch_combinatoric(int kind, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                               int tr, uint64_t total, int grid, void *partials, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)m * n * (kind == ENGINE_CPLX ? 2 : 1);
  switch (kind) {
    case ENGINE_REAL:
      hipLaunchKernelGGL(combinatoric_kernel<ENGINE_REAL>, dim3(grid), dim3(kThreads), lds, s, m,
                         n, dt, dA, lda, tr, total, partials);
      break;
    case ENGINE_CPLX:
      hipLaunchKernelGGL(combinatoric_kernel<ENGINE_CPLX>, dim3(grid), dim3(kThreads), lds, s, m,
                         n, dt, dA, lda, tr, total, partials);
      break;
    default:
      hipLaunchKernelGGL(combinatoric_kernel<ENGINE_INT>, dim3(grid), dim3(kThreads), lds, s, m,
                         n, dt, dA, lda, tr, total, partials);
      break;
  }
  return hipGetLastError();
}

}  // namespace permgpu
