// Rectangular permanent through the elementary symmetric polynomial e_m, on
// gfx950: the lane types and the walk kernel shared by the generic
// instantiations (esym.inc, one kernel per n) and the banded ones
// (esym_band.inc, one kernel per (n, m)).
//
// Glynn's formula for the square matrix A' = [A; J] padded with n - m rows of
// ones (Sec. 1.2, Eq. glynn_filled_matrix and Eq. glynn_rectangle) has n - m
// identical rows.  Summing their signs out leaves a sum over the signs of the
// m rows of A only:
//
//   per(A) = 2^-(m-1) sum_{delta in {+-1}^m, delta_1 = +1} (prod delta) e_m(c(delta)),
//   c_j(delta) = sum_i delta_i a_ij,
//
// because expanding e_m(c) = sum_{|T| = m} prod_{j in T} c_j into row choices,
// the sign sum over delta keeps exactly the products that use every row once
// (each injective map rows -> columns once, with T its image).  Cost
// 2^(m-1) terms instead of Glynn's 2^(n-1).
//
// The walk is the Gray-code walk of the engine (aligned blocks of 2^b steps,
// wave-uniform flip index and direction, closed-form seed per block, one
// scalar-loaded row per step) with v = c.  Each term evaluates the
// recurrence e_k <- e_k + c_j e_{k-1} over the columns j.  The generic lane
// runs every degree k <= min(n, 32) and picks e_m at run time; the banded
// lane (m a compile-time constant) runs only the degrees that can reach e_m.
// The sum is accumulated like the engine's (plain partial, TwoSum every 8
// terms) and reduced to one double-double per workgroup; the exact-integer
// kind keeps the degrees and the sum modulo 2^128.  One step per loop
// iteration: the recurrence is long enough that unrolling the steps would
// only grow the code.
#pragma once
#include "device_common.h"
#include "internal.h"

namespace permgpu {
namespace esym_detail {


constexpr int kEsymBlock = 256;
typedef __attribute__((address_space(4))) const double kdouble;

template <int NV>
constexpr int esym_mv() { return NV < ESYM_MAX_M ? NV : ESYM_MAX_M; }

template <int NV, int EK>
struct ELane;

template <int NV>
struct ELane<NV, 0> {
  static constexpr int MV = esym_mv<NV>();
  double v[NV];
  double s, hi, lo;
  int m;
  __device__ __forceinline__ void zero_acc() { s = hi = lo = 0.0; }
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
  __device__ __forceinline__ double esym() const {
    double e[MV + 1];
    e[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= MV; ++k) e[k] = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
#pragma unroll
      for (int k = (j + 1 < MV ? j + 1 : MV); k >= 1; --k) e[k] = __builtin_fma(v[j], e[k - 1], e[k]);
    }
    double r = e[MV];
#pragma unroll
    for (int k = MV - 1; k >= 1; --k) r = (k == m) ? e[k] : r;
    return r;
  }
  __device__ __forceinline__ void term(bool neg) {
    const double x = esym();
    s += neg ? -x : x;
  }
  __device__ __forceinline__ void flush() {
    dd_acc(hi, lo, s);
    s = 0.0;
  }
};

template <int NV>
struct ELane<NV, 1> {
  static constexpr int MV = esym_mv<NV>();
  double vr[NV], vi[NV];
  double sr, si, hr, lr, hi_, li;
  int m;
  __device__ __forceinline__ void zero_acc() { sr = si = hr = lr = hi_ = li = 0.0; }
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
  // e_k <- e_k + c_j e_{k-1} in complex arithmetic
  __device__ __forceinline__ void esym(double &xr, double &xi) const {
    double er[MV + 1], ei[MV + 1];
    er[0] = 1.0;
    ei[0] = 0.0;
#pragma unroll
    for (int k = 1; k <= MV; ++k) er[k] = ei[k] = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
#pragma unroll
      for (int k = (j + 1 < MV ? j + 1 : MV); k >= 1; --k) {
        const double ar = er[k - 1], ai = ei[k - 1];
        er[k] = __builtin_fma(vr[j], ar, __builtin_fma(-vi[j], ai, er[k]));
        ei[k] = __builtin_fma(vr[j], ai, __builtin_fma(vi[j], ar, ei[k]));
      }
    }
    xr = er[MV];
    xi = ei[MV];
#pragma unroll
    for (int k = MV - 1; k >= 1; --k) {
      xr = (k == m) ? er[k] : xr;
      xi = (k == m) ? ei[k] : xi;
    }
  }
  __device__ __forceinline__ void term(bool neg) {
    double xr, xi;
    esym(xr, xi);
    sr += neg ? -xr : xr;
    si += neg ? -xi : xi;
  }
  __device__ __forceinline__ void flush() {
    dd_acc(hr, lr, sr);
    dd_acc(hi_, li, si);
    sr = si = 0.0;
  }
};

// Exact integers: the column sums are integers below 2^53 (checked on the
// host), so they convert to int64 exactly; the degrees are kept modulo 2^128,
// a ring homomorphism, so the wrapped sum is exact whenever the true one fits.
template <int NV>
struct ELane<NV, 2> {
  static constexpr int MV = esym_mv<NV>();
  double v[NV];
  u128 acc;
  int m;
  __device__ __forceinline__ void zero_acc() { acc = 0; }
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
  // Only the degrees that can still reach e_m are updated: at column j,
  // max(1, j + 1 - (NV - m)) <= k <= min(j + 1, m).  m is the same in every
  // lane of the wave, so the tests are scalar branches around the 128-bit
  // multiply-adds they skip (about a third of them remain at 16 x 48).
  // The column sums are below 2^52 in magnitude (the pre-check), so each
  // multiply-add is e_k +- |c_j| e_(k-1): a 128 x 52-bit product in 32-bit
  // limbs (mul128x52) with the sign of c_j applied once per column.
  __device__ __forceinline__ u128 esym() const {
    const int mu = __builtin_amdgcn_readfirstlane(m);
    u128 e[MV + 1];
    e[0] = 1;
#pragma unroll
    for (int k = 1; k <= MV; ++k) e[k] = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int64_t ci = f64_to_i64_exact(v[j]);
      const uint64_t a = ci < 0 ? (uint64_t)0 - (uint64_t)ci : (uint64_t)ci;
      const u128 neg = (u128)(i128)(ci >> 63);  // all ones if c_j < 0
#pragma unroll
      for (int k = (j + 1 < MV ? j + 1 : MV); k >= 1; --k)
        if (k <= mu && k >= j + 1 - (NV - mu)) {
          uint64_t lo = (uint64_t)e[k - 1], hi = (uint64_t)(e[k - 1] >> 64);
          mul128x52(lo, hi, a);
          const u128 t = (((u128)hi << 64) | lo) ^ neg;
          e[k] += t - neg;
        }
    }
    u128 r = e[1];
#pragma unroll
    for (int k = 2; k <= MV; ++k)
      if (k == mu) r = e[k];
    return r;
  }
  __device__ __forceinline__ void term(bool neg) {
    const u128 x = esym();
    acc += neg ? (u128)0 - x : x;
  }
  __device__ __forceinline__ void flush() {}
};

__device__ __forceinline__ void esym_store_int(u128 x, void *partials) {
  __shared__ uint64_t ired[kEsymBlock / 64][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  const int width = blockDim.x < 64 ? (int)blockDim.x : 64;
  uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
  for (int off = width >> 1; off > 0; off >>= 1) {
    const uint64_t olo = shfl_xor_u64(lo, off, width), ohi = shfl_xor_u64(hi, off, width);
    const u128 y = (((u128)hi) << 64 | lo) + (((u128)ohi) << 64 | olo);
    lo = (uint64_t)y;
    hi = (uint64_t)(y >> 64);
  }
  if (lane == 0) {
    ired[wave][0] = lo;
    ired[wave][1] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u128 y = 0;
    for (int w = 0; w < nwaves; ++w) y += ((u128)ired[w][1]) << 64 | ired[w][0];
    uint64_t *p = (uint64_t *)partials + 2 * blockIdx.x;
    p[0] = (uint64_t)y;
    p[1] = (uint64_t)(y >> 64);
  }
}

// One workgroup partial: real {hi, lo}, complex {re.hi, re.lo, im.hi, im.lo}.
__device__ __forceinline__ void esym_store(int ncomp, double *x /* 2 or 4 dd words */,
                                           void *partials) {
  __shared__ double red[kEsymBlock / 64][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  const int width = blockDim.x < 64 ? (int)blockDim.x : 64;
  for (int c = 0; c < ncomp; ++c) {
    double h, l;
    fast_two_sum(x[2 * c], x[2 * c + 1], h, l);
    for (int off = width >> 1; off > 0; off >>= 1) {
      const double oh = shfl_xor_d(h, off, width), ol = shfl_xor_d(l, off, width);
      dd_add(h, l, oh, ol);
    }
    if (lane == 0) {
      red[wave][2 * c] = h;
      red[wave][2 * c + 1] = l;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double *p = (double *)partials + 2 * ncomp * blockIdx.x;
    for (int c = 0; c < ncomp; ++c) {
      double H = red[0][2 * c], L = red[0][2 * c + 1];
      for (int w = 1; w < nwaves; ++w) dd_add(H, L, red[w][2 * c], red[w][2 * c + 1]);
      p[2 * c] = H;
      p[2 * c + 1] = L;
    }
  }
}

// Registers: NV sums and MV + 1 degrees (twice for complex); long vectors run
// fewer waves per SIMD rather than spill.
template <int NV, int EK>
constexpr int esym_waves_per_eu() {
  if constexpr (EK == 1) return NV <= 12 ? 2 : 1;
  if constexpr (EK == 2) return NV <= 12 ? 2 : 1;
  return NV <= 24 ? 4 : 2;
}


// ---- exact degree m: the band of the recurrence ----
// Degree k at column j (0-based) is needed only if it can still reach e_m:
// k <= j + 1 (no more columns seen) and k >= m - (n - 1 - j) (enough columns
// left), so column j updates the degrees
//   LO(j) = max(1, j + 1 - (n - m)) .. HI(j) = min(j + 1, m),
// about m (n - m + 1) multiply-adds per term instead of n min(m, 32); the
// first touch of a degree (k = j + 1, where e_k is still 0) is a multiply,
// and degree 1 (e_0 = 1) an add.  With n and m compile-time constants the
// whole band unrolls into straight-line code over registers.
template <int J, int K, int LO>
struct BandColR {
  template <int M1>
  static __device__ __forceinline__ void run(double (&e)[M1], double c) {
    if constexpr (K >= LO) {
      if constexpr (K == J + 1) e[K] = c * e[K - 1];
      else e[K] = __builtin_fma(c, e[K - 1], e[K]);
      BandColR<J, K - 1, LO>::run(e, c);
    }
  }
};
// complex: e_k += c e_{k-1}
template <int J, int K, int LO>
struct BandColC {
  template <int M1>
  static __device__ __forceinline__ void run(double (&er)[M1], double (&ei)[M1], double cr,
                                             double ci) {
    if constexpr (K >= LO) {
      const double ar = er[K - 1], ai = ei[K - 1];
      if constexpr (K == J + 1) {
        er[K] = __builtin_fma(cr, ar, -(ci * ai));
        ei[K] = __builtin_fma(cr, ai, ci * ar);
      } else {
        er[K] = __builtin_fma(cr, ar, __builtin_fma(-ci, ai, er[K]));
        ei[K] = __builtin_fma(cr, ai, __builtin_fma(ci, ar, ei[K]));
      }
      BandColC<J, K - 1, LO>::run(er, ei, cr, ci);
    }
  }
};
template <int NV, int M, int J>
struct BandCols {
  static constexpr int D = NV - M;
  static constexpr int LO = (J + 1 - D) > 1 ? (J + 1 - D) : 1;
  static constexpr int HI = (J + 1) < M ? (J + 1) : M;
  static __device__ __forceinline__ void real(double (&e)[M + 1], const double (&v)[NV]) {
    if constexpr (J < NV) {
      BandColR<J, HI, LO>::run(e, v[J]);
      BandCols<NV, M, J + 1>::real(e, v);
    }
  }
  static __device__ __forceinline__ void cplx(double (&er)[M + 1], double (&ei)[M + 1],
                                              const double (&vr)[NV], const double (&vi)[NV]) {
    if constexpr (J < NV) {
      BandColC<J, HI, LO>::run(er, ei, vr[J], vi[J]);
      BandCols<NV, M, J + 1>::cplx(er, ei, vr, vi);
    }
  }
};

// Multiply-adds of the band per term (the algorithmic count of one term's
// recurrence; real kind, one VALU operation each).
__host__ __device__ constexpr int esym_band_ops(int nv, int m) {
  int ops = 0;
  for (int j = 0; j < nv; ++j) {
    const int lo = (j + 1 - (nv - m)) > 1 ? (j + 1 - (nv - m)) : 1;
    const int hi = (j + 1) < m ? (j + 1) : m;
    if (hi >= lo) ops += hi - lo + 1;
  }
  return ops;
}

template <int NV, int M, int EK>
struct BLane;

// Waves per SIMD for a banded kernel: registers for the NV sums, the live
// band of degrees (at most min(m, n - m + 1) + 1) and temporaries, out of 512.
template <int NV, int M, int EK>
constexpr int esym_band_waves_per_eu() {
  constexpr int w = (M < NV - M + 1 ? M : NV - M + 1) + 2;
  constexpr int need = (EK == 1 ? 2 : 1) * (2 * NV + 2 * w) + 16;
  constexpr int wpe = 512 / need;
  return wpe < 1 ? 1 : (wpe > 4 ? 4 : wpe);
}

template <int NV, int M>
struct BLane<NV, M, 0> : ELane<NV, 0> {
  __device__ __forceinline__ void term(bool neg) {
    double e[M + 1];
    e[0] = 1.0;
    BandCols<NV, M, 0>::real(e, this->v);
    this->s += neg ? -e[M] : e[M];
  }
};

template <int NV, int M>
struct BLane<NV, M, 1> : ELane<NV, 1> {
  __device__ __forceinline__ void term(bool neg) {
    double er[M + 1], ei[M + 1];
    er[0] = 1.0;
    ei[0] = 0.0;
    BandCols<NV, M, 0>::cplx(er, ei, this->vr, this->vi);
    this->sr += neg ? -er[M] : er[M];
    this->si += neg ? -ei[M] : ei[M];
  }
};

// The walk over the signs of rows 1..m-1 (Gray order, aligned blocks of 2^b
// steps, closed-form seed per block), one e_m term per step.  LaneT is the
// generic lane (ELane: degrees up to min(n, 32), e_m picked at run time) or
// the banded one (BLane: exact m).
template <class LaneT, int NV, int EK, int WPE>
__global__ __launch_bounds__(kEsymBlock, WPE) void esym_walk_kernel(GrayWalk w, void *partials) {
  constexpr int C = EK == 1 ? 2 : 1;
  auto row = [](const double *__restrict__ t, int q, uint32_t d) {
    asm volatile("" : "+s"(t));
    return (const kdouble *)(t + (size_t)(2 * q + (int)d) * NV * C);
  };
  const double *__restrict__ tbl = w.tbl;
  const int b = w.b;
  const uint32_t B = 1u << b;
  const uint64_t lanes = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gl = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int qstart = b > 0 ? b - 1 : 0;

  LaneT L;
  L.zero_acc();
  L.m = w.m;
  for (uint64_t r = 0; r < w.blocks_per_lane; ++r) {
    // block index with the same parity in every lane (as in the engine)
    const uint64_t blk = w.blocks_per_lane == 1 ? gl : ((((r >> 1) * lanes + gl) << 1) | (r & 1));
    const uint64_t k0 = blk << b;
    const uint32_t kpar = (uint32_t)(r & 1) << b;
    L.load_base(w.base);
    const uint64_t g0 = k0 ^ (k0 >> 1);
    for (int q = qstart; q < w.nbits; ++q) L.seed_add(tbl + (size_t)(2 * q) * NV * C, (double)((g0 >> q) & 1u));
    // the first term's sign is the parity of k0 (odd only for one-term
    // blocks, b = 0); the flips inside a block alternate it
    L.term((k0 & 1u) != 0);
    for (uint32_t t = 1; t < B; ++t) {
      const int q = __builtin_ctz(t);
      L.apply(row(tbl, q, ((kpar + t) >> (q + 1)) & 1u));
      L.term((t & 1u) != 0);
      if ((t & 7u) == 7u) L.flush();
    }
    L.flush();
  }
  if constexpr (EK == 2) {
    esym_store_int(L.acc, partials);
  } else if constexpr (EK == 1) {
    double x[4] = {L.hr, L.lr, L.hi_, L.li};
    esym_store(2, x, partials);
  } else {
    double x[2] = {L.hi, L.lo};
    esym_store(1, x, partials);
  }
}

}  // namespace esym_detail
}  // namespace permgpu
