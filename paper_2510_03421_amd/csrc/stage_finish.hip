// Staging of the input into Gray-walk update tables, the deterministic final
// reduction with the per-algorithm normalisation, and the absolute-sum pass of
// the integer overflow pre-check.
#include "device_common.h"
#include "finish_common.h"
#include "input_read.h"
#include "internal.h"
#include "pad_model.h"

namespace permgpu {
namespace {

// Exponent e of the padding value 2^e of the floating-point Glynn sum on an
// m x n matrix (m < n), chosen by pad_exponent from the data's mean square.
// One workgroup; the result goes to *e (0 for a zero matrix).
__global__ __launch_bounds__(kReduceThreads) void pad_scale_kernel(int m, int n, perm_dtype dt,
                                                                  const void *dA, int64_t lda,
                                                                  int tr, int *e) {
  __shared__ double sh[kReduceThreads];
  __shared__ float f[kPadScratch];
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < m * n; idx += blockDim.x) {
    double re, im;
    read_entry(dt, dA, lda, tr, idx / n, idx % n, re, im);
    acc += re * re + im * im;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const int x = pad_exponent(m, n, sh[0], (int)threadIdx.x, (int)blockDim.x, f);
  if (threadIdx.x == 0) *e = x;
}

// algo 0 (Glynn): NV = n, nbits = n-1, padded matrix a' (rows m..n-1 hold the
//   padding value: 2^(*pad_exp), or 1 when pad_exp is null),
//   base_j = sum_i a'_ij, U[q]_j = -2 a'_{q+1, j}.
// algo 1 (square Ryser): NV = m, nbits = n, base = 0, U[q]_i = a_{i, q}.
// algo 2 (signs of the m rows only, no padding): NV = n, nbits = m-1,
//   base_j = sum_{i<m} a_ij, U[q]_j = -2 a_{q+1, j}.
// A chunk of the walk -- the indices K0 + k, K0 = c 2^B, k < 2^B -- is the
// walk over the low B bits: g(K0 + k) = g(K0) xor g(k), so it starts from
// v(K0) = base + sum over the set bits q of g_start = g(K0) of U[q], and
// every row whose bit is set in g_start enters the table with the opposite
// sign (the chunk walk uses the rows q < B, where only q = B-1 can be set,
// for odd c).  g_start = 0 is the whole walk.
__device__ __forceinline__ void update_entry(int algo, int m, perm_dtype dt, const void *dA,
                                             int64_t lda, int tr, double pad, int q, int j,
                                             double &re, double &im,
                                             const int32_t *col_order = nullptr) {
  if (algo != 1) {
    if (q + 1 < m) {
      read_entry(dt, dA, lda, tr, q + 1, j, re, im);
    } else {
      re = pad;
      im = 0.0;
    }
    re *= -2.0;
    im *= -2.0;
  } else {
    read_entry(dt, dA, lda, tr, j, col_order ? col_order[q] : q, re, im);
  }
}

__global__ void stage_gray_kernel(int algo, int m, int n, perm_dtype dt, const void *dA,
                                  int64_t lda, int tr, double *tbl, double *base, int C,
                                  const int *pad_exp, uint64_t g_start,
                                  const int32_t *col_order) {
  const double pad = pad_exp ? __builtin_ldexp(1.0, *pad_exp) : 1.0;
  const int nv = algo == 1 ? m : n;
  const int nbits = algo == 0 ? n - 1 : (algo == 1 ? n : m - 1);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < nbits * nv) {
    const int q = idx / nv, j = idx % nv;
    double re, im;
    update_entry(algo, m, dt, dA, lda, tr, pad, q, j, re, im, col_order);
    if ((g_start >> q) & 1u) {
      re = -re;
      im = -im;
    }
    double *p = tbl + (size_t)(2 * q) * nv * C + (size_t)j * C;
    double *mneg = tbl + (size_t)(2 * q + 1) * nv * C + (size_t)j * C;
    p[0] = re;
    mneg[0] = -re;
    if (C == 2) {
      p[1] = im;
      mneg[1] = -im;
    }
  }
  if (idx < nv) {
    double sr = 0.0, si = 0.0;
    if (algo != 1) {
      for (int i = 0; i < (algo == 0 ? n : m); ++i) {
        double re = pad, im = 0.0;
        if (i < m) read_entry(dt, dA, lda, tr, i, idx, re, im);
        sr += re;
        si += im;
      }
    }
    for (int q = 0; q < nbits; ++q) {
      if ((g_start >> q) & 1u) {
        double re, im;
        update_entry(algo, m, dt, dA, lda, tr, pad, q, idx, re, im, col_order);
        sr += re;
        si += im;
      }
    }
    base[(size_t)idx * C] = sr;
    if (C == 2) base[(size_t)idx * C + 1] = si;
  }
}

// Walks of fewer than 8 terms (nbits <= 2: Glynn n <= 3, square Ryser
// n <= 2, chunks of 2 or 4 indices), which the block engine does not take.
// One wave: lane k < 2^nbits forms v(k) = base + sum over the set bits q of
// g(k) of U[q] column by column and multiplies the entries into its term;
// lane 0 adds the signed terms in index order into partial slot 0 (format of
// the engine's partials).  Integer products are exact (every |v_j| < 2^53 by
// the pre-check) and taken modulo 2^128.
__global__ __launch_bounds__(64) void gray_tiny_kernel(int kind, const double *tbl,
                                                      const double *base, int nv, int nbits,
                                                      void *partials) {
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  const int k = threadIdx.x;
  const int terms = 1 << nbits;
  __shared__ double tr_[8], ti_[8];
  __shared__ uint64_t tlo[8], thi[8];
  if (k < terms) {
    const uint32_t g = (uint32_t)(k ^ (k >> 1));
    double pr = 1.0, pi = 0.0;
    u128 pint = 1;
    for (int j = 0; j < nv; ++j) {
      double vr = base[(size_t)j * C], vi = C == 2 ? base[(size_t)j * C + 1] : 0.0;
      for (int q = 0; q < nbits; ++q) {
        if ((g >> q) & 1u) {
          vr += tbl[(size_t)(2 * q) * nv * C + (size_t)j * C];
          if (C == 2) vi += tbl[(size_t)(2 * q) * nv * C + (size_t)j * C + 1];
        }
      }
      if (kind == ENGINE_INT) {
        pint *= (u128)(i128)f64_to_i64_exact(vr);
      } else if (C == 2) {
        double cr, ci;
        cmul(pr, pi, vr, vi, cr, ci);
        pr = cr;
        pi = ci;
      } else {
        pr *= vr;
      }
    }
    if (k & 1) {
      pr = -pr;
      pi = -pi;
      pint = (u128)0 - pint;
    }
    tr_[k] = pr;
    ti_[k] = pi;
    tlo[k] = (uint64_t)pint;
    thi[k] = (uint64_t)(pint >> 64);
  }
  __syncthreads();
  if (k == 0) {
    if (kind == ENGINE_INT) {
      u128 acc = 0;
      for (int i = 0; i < terms; ++i) acc += ((u128)thi[i]) << 64 | tlo[i];
      ((uint64_t *)partials)[0] = (uint64_t)acc;
      ((uint64_t *)partials)[1] = (uint64_t)(acc >> 64);
    } else {
      double rh = 0.0, rl = 0.0, ih = 0.0, il = 0.0;
      for (int i = 0; i < terms; ++i) {
        dd_add(rh, rl, tr_[i], 0.0);
        dd_add(ih, il, ti_[i], 0.0);
      }
      double *p = (double *)partials;
      p[0] = rh;
      p[1] = rl;
      if (C == 2) {
        p[2] = ih;
        p[3] = il;
      }
    }
  }
}

// ---- final reduction (one workgroup of kReduceThreads) ----
__global__ __launch_bounds__(kReduceThreads) void finish_kernel(int kind, const void *partials,
                                                                int count, Finish f, void *out) {
  __shared__ double sh[kReduceThreads][4];
  __shared__ uint64_t si[kReduceThreads][2];
  const int t = threadIdx.x;
  if (kind == ENGINE_INT) {
    u128 x = 0;
    const uint64_t *p = (const uint64_t *)partials;
    for (int i = t; i < count; i += kReduceThreads) x += ((u128)p[2 * i + 1]) << 64 | p[2 * i];
    si[t][0] = (uint64_t)x;
    si[t][1] = (uint64_t)(x >> 64);
    __syncthreads();
    for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
      if (t < off) {
        u128 a = ((u128)si[t][1]) << 64 | si[t][0];
        u128 b = ((u128)si[t + off][1]) << 64 | si[t + off][0];
        a += b;
        si[t][0] = (uint64_t)a;
        si[t][1] = (uint64_t)(a >> 64);
      }
      __syncthreads();
    }
    if (t == 0) {
      const u128 E = ((u128)si[0][1]) << 64 | si[0][0];
      write_int(f.ot, int_per(E, f.mode, f.m, f.n), out, 0);
    }
    return;
  }
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  const double *p = (const double *)partials;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int i = t; i < count; i += kReduceThreads) {
    dd_add(a, b, p[2 * C * i], p[2 * C * i + 1]);
    if (C == 2) dd_add(c, d, p[4 * i + 2], p[4 * i + 3]);
  }
  sh[t][0] = a; sh[t][1] = b; sh[t][2] = c; sh[t][3] = d;
  __syncthreads();
  for (int off = kReduceThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      dd_add(sh[t][0], sh[t][1], sh[t + off][0], sh[t + off][1]);
      dd_add(sh[t][2], sh[t][3], sh[t + off][2], sh[t + off][3]);
    }
    __syncthreads();
  }
  if (t == 0) {
    double rh = sh[0][0], rl = sh[0][1], ih = sh[0][2], il = sh[0][3];
    fp_per(f.mode, f.m, f.n, f.pad_exp ? *f.pad_exp : 0, C == 2, rh, rl, ih, il);
    write_fp(f.ot, rh, rl, ih, il, out, 0);
  }
}

// Per-line magnitudes of an integer matrix.  mode 0: absolute sum of each
// logical row, 1: of each column (exact in 64 bits, saturating); mode 2 / 3:
// sum of squares of each row / column as a double (bit pattern in the slot).
// One thread per logical row (idx < m) or column (idx = m + j) of an integer
// matrix: its absolute sum (exact, saturating at 2^64 - 1) and its sum of
// squares (a double's bit pattern); a row also gets the bit mask of its
// nonzero entries (columns below 64).  Layout of `out`: abs[m + n],
// sq[m + n], masks[m].
__global__ void int_stats_kernel(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                                 uint64_t *out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m + n) return;
  const bool col = idx >= m;
  const int len = col ? m : n;
  u128 s = 0;
  double q = 0.0;
  uint64_t mask = 0;
  for (int k = 0; k < len; ++k) {
    const int i = col ? k : idx, j = col ? idx - m : k;
    const int64_t o = tr ? (int64_t)j * lda + i : (int64_t)i * lda + j;
    int64_t x;
    if (dt == PERM_I64) x = ((const int64_t *)dA)[o];
    else x = ((const uint8_t *)dA)[o] ? 1 : 0;
    s += x < 0 ? (u128)(-(i128)x) : (u128)x;
    const double xd = (double)x;
    q = __builtin_fma(xd, xd, q);
    if (x != 0 && k < 64) mask |= 1ull << k;
  }
  out[idx] = (s >> 64) ? ~0ull : (uint64_t)s;
  out[m + n + idx] = (uint64_t)__double_as_longlong(q);
  if (!col) out[2 * (m + n) + idx] = mask;
}

__global__ void write_one_kernel(perm_out ot, void *out) {
  switch (ot) {
    case PERM_OUT_F64: ((double *)out)[0] = 1.0; break;
    case PERM_OUT_DD: ((double *)out)[0] = 1.0; ((double *)out)[1] = 0.0; break;
    case PERM_OUT_C128: ((double *)out)[0] = 1.0; ((double *)out)[1] = 0.0; break;
    case PERM_OUT_CDD:
      ((double *)out)[0] = 1.0;
      ((double *)out)[1] = ((double *)out)[2] = ((double *)out)[3] = 0.0;
      break;
    case PERM_OUT_I64: ((int64_t *)out)[0] = 1; break;
    default: ((uint64_t *)out)[0] = 1; ((uint64_t *)out)[1] = 0; break;
  }
}

// D[(out * l + in)] = col[in] - col[out] over the low columns
__global__ void stage_rect_kernel(int m, int n, int l, perm_dtype dt, const void *dA, int64_t lda,
                                  int tr, double *colT, double *D, int C) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  auto rd = [&](int i, int j, double &re, double &im) {
    const int64_t o = tr ? (int64_t)j * lda + i : (int64_t)i * lda + j;
    im = 0.0;
    switch (dt) {
      case PERM_F64: re = ((const double *)dA)[o]; break;
      case PERM_C128:
        re = ((const double *)dA)[2 * o];
        im = ((const double *)dA)[2 * o + 1];
        break;
      case PERM_I64: re = (double)((const int64_t *)dA)[o]; break;
      default: re = ((const uint8_t *)dA)[o] ? 1.0 : 0.0; break;
    }
  };
  if (idx < n * m) {
    const int j = idx / m, i = idx % m;
    double re, im;
    rd(i, j, re, im);
    colT[((size_t)j * m + i) * C] = re;
    if (C == 2) colT[((size_t)j * m + i) * C + 1] = im;
  }
  if (idx < l * l * m) {
    const int pair = idx / m, i = idx % m;
    const int out = pair / l, in = pair % l;
    double ro, io, rn, in_;
    rd(i, out, ro, io);
    rd(i, in, rn, in_);
    D[((size_t)pair * m + i) * C] = rn - ro;
    if (C == 2) D[((size_t)pair * m + i) * C + 1] = in_ - io;
  }
}

}  // namespace

hipError_t launch_pad_scale(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                            int *e, hipStream_t s) {
  hipLaunchKernelGGL(pad_scale_kernel, dim3(1), dim3(kReduceThreads), 0, s, m, n, dt, dA, lda, tr,
                     e);
  return hipGetLastError();
}

hipError_t launch_stage_gray(int algo, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                             int tr, double *tbl, double *base, int cplx, hipStream_t s,
                             const int *pad_exp, uint64_t g_start, const int32_t *col_order) {
  const int nv = algo == 1 ? m : n;
  const int nbits = algo == 0 ? n - 1 : (algo == 1 ? n : m - 1);
  int work = nbits * nv > nv ? nbits * nv : nv;
  if (work < 1) work = 1;
  const int threads = 256, blocks = (work + threads - 1) / threads;
  hipLaunchKernelGGL(stage_gray_kernel, dim3(blocks), dim3(threads), 0, s, algo, m, n, dt, dA, lda,
                     tr, tbl, base, cplx ? 2 : 1, pad_exp, g_start, col_order);
  return hipGetLastError();
}


hipError_t launch_gray_tiny(int kind, const GrayWalk &w, void *partials, hipStream_t s) {
  hipLaunchKernelGGL(gray_tiny_kernel, dim3(1), dim3(64), 0, s, kind, w.tbl, w.base, w.nv, w.nbits,
                     partials);
  return hipGetLastError();
}

hipError_t launch_finish(int kind, const void *partials, int count, const Finish &f, void *dOut,
                         hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kReduceThreads), 0, s, kind, partials, count, f,
                     dOut);
  return hipGetLastError();
}

// one thread per row: the bit mask of its nonzero entries (real or complex)
__global__ void row_masks_kernel(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                                 uint64_t *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint64_t mask = 0;
  for (int j = 0; j < n && j < 64; ++j) {
    double re, im;
    read_entry(dt, dA, lda, tr, i, j, re, im);
    if (re != 0.0 || im != 0.0) mask |= 1ull << j;
  }
  out[i] = mask;
}

hipError_t launch_row_masks(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                            uint64_t *out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_masks_kernel, dim3((m + 63) / 64), dim3(64), 0, s, m, n, dt, dA, lda, tr,
                     out);
  return hipGetLastError();
}

hipError_t launch_int_stats(int m, int n, perm_dtype dt, const void *dA, int64_t lda, int tr,
                            uint64_t *out, hipStream_t s) {
  const int count = m + n;
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(int_stats_kernel, dim3((count + 63) / 64), dim3(64), 0, s, m, n, dt, dA, lda,
                     tr, out);
  return hipGetLastError();
}

hipError_t launch_stage_rect(int m, int n, int l, perm_dtype dt, const void *dA, int64_t lda,
                             int tr, double *colT, double *D, int cplx, hipStream_t s) {
  int work = n * m > l * l * m ? n * m : l * l * m;
  if (work < 1) work = 1;
  hipLaunchKernelGGL(stage_rect_kernel, dim3((work + 255) / 256), dim3(256), 0, s, m, n, l, dt, dA,
                     lda, tr, colT, D, cplx ? 2 : 1);
  return hipGetLastError();
}

hipError_t launch_ryser_rect(int kind, const RectWalk &w, int grid, void *partials,
                             hipStream_t s) {
  switch (kind) {
    case ENGINE_REAL: return launch_ryser_rect_real(w, grid, partials, s);
    case ENGINE_CPLX: return launch_ryser_rect_cplx(w, grid, partials, s);
    default: return launch_ryser_rect_int(w, grid, partials, s);
  }
}

hipError_t launch_write_one(perm_out ot, void *dOut, hipStream_t s) {
  hipLaunchKernelGGL(write_one_kernel, dim3(1), dim3(1), 0, s, ot, dOut);
  return hipGetLastError();
}

}  // namespace permgpu
