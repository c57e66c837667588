// Gray-code walks of small square matrices in one workgroup: Glynn's formula
// (Sec. 1.2 Eq. glynn) over n - 1 sign bits or Ryser's (Eq. ryser_square)
// over n subset bits, at most 2^15 terms.  The whole call is one launch: the
// workgroup stages the update table in LDS (rows padded to 16 entries with
// zeros, the start vector with ones, so every product runs over 16 factors
// and the padding multiplies by 1), each lane walks one aligned block of
// 2^nbits / lanes consecutive Gray indices from its closed-form seed, the
// lanes' signed sums are reduced in a fixed order, and thread 0 normalises
// and writes the result.  For these sizes the multi-kernel path (staging
// kernel, engine, finishing kernel, scratch from the stream-ordered pool) is
// bound by launch latency, not by the terms.
#include "device_common.h"
#include "finish_common.h"
#include "input_read.h"
#include "internal.h"

namespace permgpu {
namespace {

// threads per workgroup: 1024 (4 waves per SIMD, 128 registers), complex
// 512 (its 2 x 16 sums and complex product chains need more registers)
template <int KIND>
constexpr int sm_threads() { return KIND == ENGINE_CPLX ? 512 : 1024; }
constexpr int kSmMaxWaves = 16;
constexpr int kSmNV = SMALL_WALK_MAX_NV;
constexpr int kSmBits = SMALL_WALK_MAX_BITS;

// thread 0 receives the workgroup's double-double sum of (h, l)
__device__ __forceinline__ void block_dd(double &h, double &l) {
  __shared__ double red[kSmMaxWaves][2];
  const int nwaves = (int)blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double a, b;
  fast_two_sum(h, l, a, b);
  for (int off = 32; off > 0; off >>= 1) {
    const double oa = shfl_xor_d(a, off, 64), ob = shfl_xor_d(b, off, 64);
    dd_add(a, b, oa, ob);
  }
  if (lane == 0) {
    red[wave][0] = a;
    red[wave][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double H = red[0][0], L = red[0][1];
    for (int w = 1; w < nwaves; ++w) dd_add(H, L, red[w][0], red[w][1]);
    h = H;
    l = L;
  }
  __syncthreads();
}

__device__ __forceinline__ u128 block_u128(u128 x) {
  __shared__ uint64_t red[kSmMaxWaves][2];
  const int nwaves = (int)blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t olo = shfl_xor_u64(lo, off, 64), ohi = shfl_xor_u64(hi, off, 64);
    const u128 y = (((u128)hi) << 64 | lo) + (((u128)ohi) << 64 | olo);
    lo = (uint64_t)y;
    hi = (uint64_t)(y >> 64);
  }
  if (lane == 0) {
    red[wave][0] = lo;
    red[wave][1] = hi;
  }
  __syncthreads();
  u128 y = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nwaves; ++w) y += ((u128)red[w][1]) << 64 | red[w][0];
  return y;
}

template <int KIND>
__global__ __launch_bounds__(sm_threads<KIND>()) void small_walk_kernel(SmallWalk a, void *out) {
  constexpr int C = KIND == ENGINE_CPLX ? 2 : 1;
  __shared__ double tbl[2 * kSmBits * kSmNV * C];  // row (q, d) at (2q + d) kSmNV C
  __shared__ double base[kSmNV * C];
  const int n = a.n;
  const int nbits = a.algo == 0 ? n - 1 : n;
  // the update table: Glynn flips row q + 1's sign (the column sums change by
  // -2 a_(q+1) j), Ryser adds column q to the row sums; d = 1 the negation
  for (int idx = threadIdx.x; idx < nbits * kSmNV; idx += blockDim.x) {
    const int q = idx / kSmNV, j = idx % kSmNV;
    double re = 0.0, im = 0.0;
    if (j < n) {
      if (a.algo == 0) {
        read_entry(a.dt, a.dA, a.lda, a.tr, q + 1, j, re, im);
        re *= -2.0;
        im *= -2.0;
      } else {
        read_entry(a.dt, a.dA, a.lda, a.tr, j, q, re, im);
      }
    }
    double *p = tbl + (size_t)(2 * q) * kSmNV * C + (size_t)j * C;
    p[0] = re;
    p[kSmNV * C] = -re;
    if constexpr (C == 2) {
      p[1] = im;
      p[kSmNV * C + 1] = -im;
    }
  }
  // start vector at Gray index 0: Glynn's column sums with every sign +1,
  // Ryser's empty row sums; padding entries 1
  if (threadIdx.x < kSmNV) {
    const int j = threadIdx.x;
    double sr = j < n ? 0.0 : 1.0, si = 0.0;
    if (j < n && a.algo == 0) {
      for (int i = 0; i < n; ++i) {
        double re, im;
        read_entry(a.dt, a.dA, a.lda, a.tr, i, j, re, im);
        sr += re;
        si += im;
      }
    }
    base[j * C] = sr;
    if constexpr (C == 2) base[j * C + 1] = si;
  }
  __syncthreads();

  constexpr int kLg = KIND == ENGINE_CPLX ? 9 : 10;
  const int lg = nbits < kLg ? nbits : kLg;  // log2 of the lanes in use
  const uint32_t lanes = 1u << lg, B = 1u << (nbits - lg);
  const uint32_t tid = threadIdx.x;
  double s = 0.0, hi = 0.0, lo = 0.0;          // real
  double sr = 0.0, si = 0.0, hr = 0.0, lr = 0.0, hm = 0.0, lm = 0.0;  // complex
  u128 acc = 0;                                 // integer
  if (tid < lanes) {
    const uint32_t k0 = tid * B;
    const uint32_t g0 = k0 ^ (k0 >> 1);
    double v[kSmNV * C];
#pragma unroll
    for (int j = 0; j < kSmNV * C; ++j) v[j] = base[j];
    for (int q = 0; q < nbits; ++q)
      if ((g0 >> q) & 1u) {
        const double *r = tbl + (size_t)(2 * q) * kSmNV * C;
#pragma unroll
        for (int j = 0; j < kSmNV * C; ++j) v[j] += r[j];
      }
    for (uint32_t t = 0; t < B; ++t) {
      if (t != 0) {
        const int q = __builtin_ctz(t);
        const uint32_t d = ((k0 + t) >> (q + 1)) & 1u;
        const double *r = tbl + (size_t)(2 * q + (int)d) * kSmNV * C;
#pragma unroll
        for (int j = 0; j < kSmNV * C; ++j) v[j] += r[j];
      }
      // the sign of Gray index k is (-1)^k
      const bool neg = ((k0 + t) & 1u) != 0;
      if constexpr (KIND == ENGINE_REAL) {
        const double p = prod_chains<kSmNV, 4>(v);
        s += neg ? -p : p;
        if ((t & 7u) == 7u) {
          dd_acc(hi, lo, s);
          s = 0.0;
        }
      } else if constexpr (KIND == ENGINE_CPLX) {
        double vr[kSmNV], vi[kSmNV];
#pragma unroll
        for (int j = 0; j < kSmNV; ++j) {
          vr[j] = v[2 * j];
          vi[j] = v[2 * j + 1];
        }
        double pr, pi;
        cprod_chains<kSmNV, 4>(vr, vi, pr, pi);
        sr += neg ? -pr : pr;
        si += neg ? -pi : pi;
        if ((t & 7u) == 7u) {
          dd_acc(hr, lr, sr);
          dd_acc(hm, lm, si);
          sr = si = 0.0;
        }
      } else {
        // one factor per chunk: every entry is below 2^52 (the pre-check)
        if (neg) int_prod_acc<kSmNV, true>(acc, v, 0, a.nonneg != 0);
        else int_prod_acc<kSmNV, false>(acc, v, 0, a.nonneg != 0);
      }
    }
  }
  const int mode = a.algo == 0 ? FINISH_GLYNN : FINISH_RYSER_SQ;
  if constexpr (KIND == ENGINE_INT) {
    const u128 E = block_u128(acc);
    if (threadIdx.x == 0) write_int(a.ot, int_per(E, mode, n, n), out, 0);
  } else if constexpr (KIND == ENGINE_CPLX) {
    dd_acc(hr, lr, sr);
    dd_acc(hm, lm, si);
    block_dd(hr, lr);
    block_dd(hm, lm);
    if (threadIdx.x == 0) {
      fp_per(mode, n, n, 0, true, hr, lr, hm, lm);
      write_fp(a.ot, hr, lr, hm, lm, out, 0);
    }
  } else {
    dd_acc(hi, lo, s);
    block_dd(hi, lo);
    if (threadIdx.x == 0) {
      double zh = 0.0, zl = 0.0;
      fp_per(mode, n, n, 0, false, hi, lo, zh, zl);
      write_fp(a.ot, hi, lo, zh, zl, out, 0);
    }
  }
}

}  // namespace

hipError_t launch_small_walk(int kind, const SmallWalk &a, void *dOut, hipStream_t s) {
  switch (kind) {
    case ENGINE_REAL:
      hipLaunchKernelGGL(small_walk_kernel<ENGINE_REAL>, dim3(1), dim3(sm_threads<ENGINE_REAL>()), 0,
                         s, a, dOut);
      break;
    case ENGINE_CPLX:
      hipLaunchKernelGGL(small_walk_kernel<ENGINE_CPLX>, dim3(1), dim3(sm_threads<ENGINE_CPLX>()), 0,
                         s, a, dOut);
      break;
    default:
      hipLaunchKernelGGL(small_walk_kernel<ENGINE_INT>, dim3(1), dim3(sm_threads<ENGINE_INT>()), 0,
                         s, a, dOut);
      break;
  }
  return hipGetLastError();
}

}  // namespace permgpu
