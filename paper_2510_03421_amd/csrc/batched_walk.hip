// Staged batch walks: the staging kernel (tables into the arena), the
// overflow pre-check of exact-integer batches, the per-matrix finish, and the
// routing of each bucket to the object that instantiates its order.
#include "batched_walk_units.h"
#include "device_common.h"
#include "finish_common.h"
#include "internal.h"

namespace permgpu {
namespace {

__device__ __forceinline__ void entry(perm_dtype dt, const void *data, int64_t idx, double &re,
                                      double &im) {
  im = 0.0;
  switch (dt) {
    case PERM_F64: re = ((const double *)data)[idx]; break;
    case PERM_C128:
      re = ((const double *)data)[2 * idx];
      im = ((const double *)data)[2 * idx + 1];
      break;
    case PERM_I64: re = (double)((const int64_t *)data)[idx]; break;
    default: re = ((const uint8_t *)data)[idx] ? 1.0 : 0.0; break;
  }
}

// One workgroup of 64 threads per staged matrix: its update table and start
// vector (the single-matrix layout) at arena + d.arena.
//   Glynn:  U[q] = -2 a'_{q+1}, a' = [A; ones], base = column sums of a';
//   Ryser:  U[q] = column q of A, base = 0;
//   e_m:    U[q] = -2 a_{q+1}, base = column sums of the m rows.
__global__ __launch_bounds__(64) void walk_stage_kernel(const WalkDesc *__restrict__ descs,
                                                        int count, perm_dtype dt,
                                                        const void *data, double *arena, int C) {
  const int i = blockIdx.x;
  if (i >= count) return;
  const WalkDesc d = descs[i];
  if (d.n == 0) return;
  double *tbl = arena + d.arena;
  double *base = tbl + (size_t)2 * d.nbits * d.nv * C;
  auto a = [&](int r, int c, double &re, double &im) {
    if (r >= d.m) {  // a padding row of ones (Glynn)
      re = 1.0;
      im = 0.0;
    } else {
      entry(dt, data, d.offset + (int64_t)r * d.ld + c, re, im);
    }
  };
  for (int idx = threadIdx.x; idx < d.nbits * d.nv; idx += 64) {
    const int q = idx / d.nv, j = idx % d.nv;
    double re, im;
    if (d.walk == WALK_RYSER) {
      a(j, q, re, im);
    } else {
      a(q + 1, j, re, im);
      re *= -2.0;
      im *= -2.0;
    }
    double *p = tbl + (size_t)(2 * q) * d.nv * C + (size_t)j * C;
    double *mneg = tbl + (size_t)(2 * q + 1) * d.nv * C + (size_t)j * C;
    p[0] = re;
    mneg[0] = -re;
    if (C == 2) {
      p[1] = im;
      mneg[1] = -im;
    }
  }
  for (int j = threadIdx.x; j < d.nv; j += 64) {
    double sr = 0.0, si = 0.0;
    if (d.walk != WALK_RYSER) {
      const int rows = d.walk == WALK_GLYNN ? d.n : d.m;
      for (int r = 0; r < rows; ++r) {
        double re, im;
        a(r, j, re, im);
        sr += re;
        si += im;
      }
    }
    base[(size_t)j * C] = sr;
    if (C == 2) base[(size_t)j * C + 1] = si;
  }
}

// Exact-integer pre-check, one thread per staged matrix (n <= 32): the
// factors' bounds (absolute row sums for Ryser, column sums for Glynn -- with
// the n - m padding ones -- and the e_m form) give the product's chunk
// selector (flag if a single factor can reach 2^52); the product
// of the absolute row sums bounds |per| (flag if the result, times 2^(n-1)
// (n-m)! for Glynn or 2^(m-1) for the e_m form, may reach 2^127, or |per|
// may reach 2^63 for 64-bit outputs; not checked under PERM_FLAG_WRAP); for
// 0/1 input Bregman's bound replaces it where smaller.
__global__ void walk_bounds_kernel(WalkDesc *descs, int count, perm_dtype dt, const void *data,
                                   perm_out ot, int wrap, int *flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  WalkDesc d = descs[i];
  if (d.n == 0) {
    flags[i] = 0;
    return;
  }
  auto absv = [&](int r, int c) -> uint64_t {
    if (r >= d.m) return 1;
    const int64_t idx = d.offset + (int64_t)r * d.ld + c;
    if (dt == PERM_I64) {
      const int64_t x = ((const int64_t *)data)[idx];
      return x < 0 ? (uint64_t)0 - (uint64_t)x : (uint64_t)x;
    }
    return ((const uint8_t *)data)[idx] ? 1 : 0;
  };
  auto sat_add = [](uint64_t a, uint64_t b) { return a > ~0ull - b ? ~0ull : a + b; };
  uint64_t bnd[32];
  const int nf = d.walk == WALK_RYSER ? d.m : d.n;
  for (int f = 0; f < nf; ++f) {
    uint64_t s = 0;
    if (d.walk == WALK_RYSER) {
      for (int c = 0; c < d.n; ++c) s = sat_add(s, absv(f, c));
    } else {
      const int rows = d.walk == WALK_GLYNN ? d.n : d.m;
      for (int r = 0; r < rows; ++r) s = sat_add(s, absv(r, f));
    }
    bnd[f] = s;
  }
  // the product's chunk selector: the fewest chunks of K = ceil(nf / NCH)
  // factors whose bound products stay below 2^52 (-1: a factor can reach it)
  const uint64_t lim = 1ull << 52;
  int pl = -1;
  bool single_ok = true;
  for (int f = 0; f < nf; ++f)
    if (bnd[f] >= lim) single_ok = false;
  for (int sel = kIntProdSelectors - 1; sel >= 0 && pl < 0 && single_ok; --sel) {
    int nch = int_chunk_count(sel, nf);
    if (nch > nf) nch = nf;
    const int c = (nf + nch - 1) / nch;
    bool ok = true;
    for (int s0 = 0; s0 < nf && ok; s0 += c) {
      u128 prod = 1;
      for (int f = s0; f < nf && f < s0 + c; ++f) {
        prod *= (u128)bnd[f];
        if (prod >= (u128)lim) break;
      }
      if (prod >= (u128)lim) ok = false;
    }
    if (ok) pl = sel;
  }
  int flag = pl < 0;
  if (!flag && !wrap) {
    double lg = 0.0;
    bool zero = false;
    for (int r = 0; r < d.m; ++r) {
      uint64_t s = 0;
      for (int c = 0; c < d.n; ++c) s = sat_add(s, absv(r, c));
      if (s == 0) zero = true;
      else lg += log2((double)s);
    }
    if (!zero && dt == PERM_B8) {
      // 0/1 input: Bregman's bound on the square 0/1 matrix [A; J] padded
      // with n - m rows of ones, per([A; J]) = (n-m)! per(A) <= prod over
      // rows of (r!)^(1/r)
      double lb = 0.0;
      for (int r = 0; r < d.m; ++r) {
        uint64_t s = 0;
        for (int c = 0; c < d.n; ++c) s = sat_add(s, absv(r, c));
        lb += lgamma((double)s + 1.0) / (double)s;
      }
      lb += (double)(d.n - d.m) * lgamma((double)d.n + 1.0) / (double)d.n;
      lb -= lgamma((double)(d.n - d.m) + 1.0);
      lb /= 0.6931471805599453;  // ln -> log2
      lg = lb < lg ? lb : lg;
    }
    if (!zero) {
      lg = lg * (1.0 + 1e-12) + 1e-9;
      if (ot == PERM_OUT_I64 && lg >= 63.0) flag = 1;
      if (lg >= 127.0) flag = 1;
      double lx = lg;
      if (d.walk == WALK_GLYNN) {
        lx += (double)(d.n - 1);
        for (int q = 2; q <= d.n - d.m; ++q) lx += log2((double)q);
      } else if (d.walk == WALK_ESYM) {
        lx += (double)(d.m - 1);
      }
      if (lx >= 127.0) flag = 1;
    }
  }
  descs[i].pl = pl < 0 ? 0 : pl;
  flags[i] = flag;
}

// One thread per staged matrix: its slots in chunk order, normalised, written
// at its place in the batch's output.
__global__ void walk_finish_kernel(int kind, const WalkDesc *__restrict__ descs,
                                   const uint32_t *__restrict__ index, int count,
                                   const double *__restrict__ slots, perm_out ot, void *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const WalkDesc d = descs[i];
  const size_t o = index[i];
  const int mode = d.walk == WALK_RYSER ? FINISH_RYSER_SQ : FINISH_GLYNN;
  // the e_m form's sum is 2^(m-1) per: Glynn's normalisation with n = m
  const int fn = d.walk == WALK_ESYM ? d.m : d.n;
  if (kind == ENGINE_INT) {
    u128 E = 0;
    for (uint32_t c = 0; c < d.nchunks; ++c) {
      const uint64_t *p = (const uint64_t *)(slots + 4 * ((size_t)d.first_slot + c));
      E += ((u128)p[1]) << 64 | p[0];
    }
    write_int(ot, d.n == 0 ? (i128)1 : int_per(E, mode, d.m, fn), out, o);
    return;
  }
  double rh = 0, rl = 0, ih = 0, il = 0;
  if (d.n == 0) {
    rh = 1.0;
  } else {
    for (uint32_t c = 0; c < d.nchunks; ++c) {
      const double *p = slots + 4 * ((size_t)d.first_slot + c);
      dd_add(rh, rl, p[0], p[1]);
      if (kind == ENGINE_CPLX) dd_add(ih, il, p[2], p[3]);
    }
    fp_per(mode, d.m, fn, 0, kind == ENGINE_CPLX, rh, rl, ih, il);
  }
  write_fp(ot, rh, rl, ih, il, out, o);
}

}  // namespace

#define WALK_DECL(k, e, lo, hi)                                                           \
  hipError_t walk_launch_##k##e##_##lo##_##hi(const WalkBucket &, const WalkLaunch &,     \
                                              hipStream_t);                               \
  int walk_occ_##k##e##_##lo##_##hi(int);
BATCH_WALK_UNITS(WALK_DECL)
#undef WALK_DECL

hipError_t launch_walk_bucket(int kind, const WalkBucket &bk, const WalkLaunch &L, hipStream_t s) {
#define WALK_LAUNCH(k, e, lo, hi) \
  if (kind == k && bk.esym == e && bk.nv >= lo && bk.nv <= hi) return walk_launch_##k##e##_##lo##_##hi(bk, L, s);
  BATCH_WALK_UNITS(WALK_LAUNCH)
#undef WALK_LAUNCH
  return hipErrorInvalidValue;
}

int walk_blocks_per_cu(int kind, int esym, int nv) {
#define WALK_OCC(k, e, lo, hi) \
  if (kind == k && esym == e && nv >= lo && nv <= hi) return walk_occ_##k##e##_##lo##_##hi(nv);
  BATCH_WALK_UNITS(WALK_OCC)
#undef WALK_OCC
  return 0;
}

hipError_t launch_walk_bounds(const WalkLaunch &L, int *flags, int wrap, hipStream_t s) {
  if (L.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(walk_bounds_kernel, dim3((L.count + 63) / 64), dim3(64), 0, s, L.descs,
                     L.count, L.dt, L.data, L.ot, wrap, flags);
  return hipGetLastError();
}

hipError_t launch_walk_batch(const WalkLaunch &L, hipStream_t s) {
  if (L.count <= 0) return hipSuccess;
  const int C = L.kind == ENGINE_CPLX ? 2 : 1;
  hipLaunchKernelGGL(walk_stage_kernel, dim3(L.count), dim3(64), 0, s, L.descs, L.count, L.dt,
                     L.data, L.arena, C);
  hipError_t e = hipGetLastError();
  for (int i = 0; i < L.nbuckets && e == hipSuccess; ++i)
    e = launch_walk_bucket(L.kind, L.buckets[i], L, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(walk_finish_kernel, dim3((L.count + 255) / 256), dim3(256), 0, s, L.kind,
                     L.descs, L.index, L.count, (const double *)L.slots, L.ot, L.out);
  return hipGetLastError();
}

}  // namespace permgpu
