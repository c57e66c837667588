// The definition on the GPU (Sec. 1.1 Eq. rectangular_permanent_definition;
// cost m n!/(n-m)!, Sec. 1.2): one product per injective map s:[m]->[n].
//
// Maps are ranked in lexicographic order of (s(0), ..., s(m-1)): the rank's
// mixed-radix digits d_i in bases n, n-1, ..., n-m+1 pick s(i) as the d_i-th
// column not used by rows 0..i-1.  A map splits into a prefix (rows 0..q-1)
// and a suffix (rows q..m-1); the host picks q so that there are several
// prefixes per lane.  Lane t takes the prefixes t, t + T, t + 2T, ... (T
// lanes in all), decodes each once and then walks all its suffixes in
// lexicographic order like an odometer.  Every lane walks the same suffix
// ranks in the same order, so the highest digit that changes from one map to
// the next is the same across the wave: the rows below it keep their columns
// and prefix products, and only the rows from it on get new columns -- the
// next free column above the old one at that digit, the lowest free column
// after it -- and new prefix products (the same left-to-right products as a
// fresh evaluation).  The number of rows m is a template parameter
// (n!/(n-m)! <= 2^40 forces m <= 14), so the per-row state stays in
// registers.  A is staged in LDS.  Real products are summed in plain partial
// sums of 8 maps folded into a compensated accumulator, integer products
// modulo 2^128.
#include <utility>

#include "device_common.h"
#include "internal.h"

namespace permgpu {
namespace {

constexpr int kThreads = 256;

template <typename W>
__device__ __forceinline__ int nth_unused(W used, int d) {
  // index of the d-th zero bit of `used` (0-based)
  int j = 0;
  for (;; ++j) {
    if (!((used >> j) & 1u)) {
      if (d == 0) return j;
      --d;
    }
  }
}

// lowest set bit of a nonzero mask
__device__ __forceinline__ int low_bit(uint32_t x) { return __builtin_ctz(x); }
__device__ __forceinline__ int low_bit(uint64_t x) { return __builtin_ctzll(x); }

// Column sets are bit masks of type W: 32 bits when n <= 32, else 64 (then
// m <= 8, since n!/(n-m)! <= 2^40).
template <int KIND, int M, typename W>
__global__ __launch_bounds__(kThreads) void combinatoric_kernel(int n, perm_dtype dt,
                                                                const void *dA, int64_t lda,
                                                                int tr, int q, uint64_t prefixes,
                                                                uint64_t suffixes, uint32_t rounds,
                                                                void *partials) {
  static_assert(M >= 1 && M <= 14, "the suffix step below handles rows 0..13");
  extern __shared__ double sa[];  // M*n (x2 for complex) entries
  constexpr int m = M;
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
  constexpr int kBits = 8 * (int)sizeof(W);
  const W free_cols = n >= kBits ? (W)~(W)0 : (W)(((W)1 << n) - 1);
  double hi = 0.0, lo = 0.0, hi2 = 0.0, lo2 = 0.0;
  double sr = 0.0, si = 0.0;  // plain partial sums of up to 8 maps
  u128 acc = 0;
  int col[M];
  W used[M + 1];  // columns taken by rows 0..i-1
  double pr[M], pi_[M];  // prefix products (real / complex)
  u128 pint[M];          // prefix products (integer)
  // the row-i prefix product from row i-1's and entry (i, col[i])
  auto extend = [&](int i) {
    const int j = col[i];
    if constexpr (KIND == ENGINE_REAL) {
      pr[i] = i == 0 ? sa[i * n + j] : pr[i - 1] * sa[i * n + j];
    } else if constexpr (KIND == ENGINE_CPLX) {
      const double ar = sa[2 * (i * n + j)], ai = sa[2 * (i * n + j) + 1];
      if (i == 0) {
        pr[0] = ar;
        pi_[0] = ai;
      } else {
        pr[i] = pr[i - 1] * ar - pi_[i - 1] * ai;
        pi_[i] = pr[i - 1] * ai + pi_[i - 1] * ar;
      }
    } else {
      const u128 v = (u128)(i128)__double_as_longlong(sa[i * n + j]);
      pint[i] = i == 0 ? v : pint[i - 1] * v;
    }
  };
  auto flush = [&]() {
    if constexpr (KIND != ENGINE_INT) {
      dd_acc(hi, lo, sr);
      if (C == 2) dd_acc(hi2, lo2, si);
      sr = si = 0.0;
    }
  };
  for (uint32_t k = 0; k < rounds; ++k) {
    const uint64_t pfx = (uint64_t)k * T + t;
    const bool live = pfx < prefixes;  // only the last round has lanes without a prefix
    const double lf = live ? 1.0 : 0.0;
    // prefix digits, the last prefix row least significant; then every
    // suffix row at digit 0 (the lowest free column)
    int dig[M];
    uint64_t x = live ? pfx : 0;
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
      dig[i] = 0;
      if (i < q) {
        const uint64_t base = (uint64_t)(n - i);
        dig[i] = (int)(x % base);
        x /= base;
      }
    }
    used[0] = 0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      col[i] = i < q ? nth_unused(used[i], dig[i]) : low_bit((W)(~used[i] & free_cols));
      used[i + 1] = used[i] | ((W)1 << col[i]);
      extend(i);
    }
    // the suffix odometer: its digits are the same in every lane
    int sd[M];
#pragma unroll
    for (int i = 0; i < M; ++i) sd[i] = 0;
    // runs of up to 8 maps in plain partial sums, then one compensated fold
    for (uint64_t r = 0; r < suffixes;) {
      const uint64_t run_end = r + 8 < suffixes ? r + 8 : suffixes;
      for (;;) {
        if constexpr (KIND == ENGINE_REAL) {
          sr = __builtin_fma(lf, pr[M - 1], sr);
        } else if constexpr (KIND == ENGINE_CPLX) {
          sr = __builtin_fma(lf, pr[M - 1], sr);
          si = __builtin_fma(lf, pi_[M - 1], si);
        } else {
          if (live) acc += pint[M - 1];
        }
        if (++r >= suffixes) break;
        // p = the highest suffix digit that changes (r < suffixes, so one does)
        int p = M;
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
          if (p == M && i >= q) {
            if (sd[i] + 1 == n - i) {
              sd[i] = 0;
            } else {
              ++sd[i];
              p = i;
            }
          }
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
          if (i >= p) {
            // digit p moved to the next free column above its old one; every
            // later digit restarted at 0: the lowest free column
            W avail = (W)(~used[i] & free_cols);
            if (i == p) avail &= col[i] + 1 >= kBits ? (W)0 : (W)((W)~(W)0 << (col[i] + 1));
            col[i] = low_bit(avail);
            used[i + 1] = used[i] | ((W)1 << col[i]);
            extend(i);
          }
        }
        if (r >= run_end) break;
      }
      flush();
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

constexpr int kWideMaxM = 8;  // n > 32 columns: n!/(n-m)! <= 2^40 leaves m <= 8

template <int KIND, int M>
hipError_t launch_one(int n, perm_dtype dt, const void *dA, int64_t lda, int tr, const CombPlan &c,
                      void *partials, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)M * n * (KIND == ENGINE_CPLX ? 2 : 1);
  if (n <= 32) {
    hipLaunchKernelGGL((combinatoric_kernel<KIND, M, uint32_t>), dim3(c.grid), dim3(kThreads), lds,
                       s, n, dt, dA, lda, tr, c.q, c.prefixes, c.suffixes, c.rounds, partials);
  } else if constexpr (M <= kWideMaxM) {
    hipLaunchKernelGGL((combinatoric_kernel<KIND, M, uint64_t>), dim3(c.grid), dim3(kThreads), lds,
                       s, n, dt, dA, lda, tr, c.q, c.prefixes, c.suffixes, c.rounds, partials);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KIND, int M>
int occupancy_one(int n) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  if (n <= 32)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, combinatoric_kernel<KIND, M, uint32_t>,
                                                     kThreads, 0);
  else if constexpr (M <= kWideMaxM)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, combinatoric_kernel<KIND, M, uint64_t>,
                                                     kThreads, 0);
  return e == hipSuccess ? nb : 0;
}

template <int KIND, int... Ms>
hipError_t launch_m(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                    const CombPlan &c, void *partials, hipStream_t s,
                    std::integer_sequence<int, Ms...>) {
  hipError_t e = hipErrorInvalidValue;
  ((m == Ms + 1 ? (e = launch_one<KIND, Ms + 1>(n, dt, dA, lda, tr, c, partials, s), 0) : 0),
   ...);
  return e;
}

template <int KIND, int... Ms>
int occupancy_m(int m, int n, std::integer_sequence<int, Ms...>) {
  int r = 0;
  ((m == Ms + 1 ? (r = occupancy_one<KIND, Ms + 1>(n), 0) : 0), ...);
  return r;
}

constexpr int kCombMaxM = 14;  // n!/(n-m)! >= m!, and the host limits the maps to 2^40 < 15!

}  // namespace

hipError_t launch_combinatoric(int kind, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                               int tr, const CombPlan &c, void *partials, hipStream_t s) {
  if (m < 1 || m > kCombMaxM || c.q < 0 || c.q > m) return hipErrorInvalidValue;
  const auto seq = std::make_integer_sequence<int, kCombMaxM>{};
  switch (kind) {
    case ENGINE_REAL: return launch_m<ENGINE_REAL>(m, n, dt, dA, lda, tr, c, partials, s, seq);
    case ENGINE_CPLX: return launch_m<ENGINE_CPLX>(m, n, dt, dA, lda, tr, c, partials, s, seq);
    default: return launch_m<ENGINE_INT>(m, n, dt, dA, lda, tr, c, partials, s, seq);
  }
}

int combinatoric_blocks_per_cu(int kind, int m, int n) {
  if (m < 1 || m > kCombMaxM) return 0;
  const auto seq = std::make_integer_sequence<int, kCombMaxM>{};
  switch (kind) {
    case ENGINE_REAL: return occupancy_m<ENGINE_REAL>(m, n, seq);
    case ENGINE_CPLX: return occupancy_m<ENGINE_CPLX>(m, n, seq);
    default: return occupancy_m<ENGINE_INT>(m, n, seq);
  }
}

}  // namespace permgpu
