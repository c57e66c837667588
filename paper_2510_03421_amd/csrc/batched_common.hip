// Batched Glynn: the padding exponents of rectangular matrices, the launch
// sequence (one kernel per matrix order -- packed small orders or chunked
// persistent ones -- then the finish) and the per-matrix finishing kernel.
#include "device_common.h"
#include "internal.h"
#include "pad_model.h"

namespace permgpu {
namespace {

// per rectangular matrix (one wave each): the padding exponent, chosen by
// pad_exponent from the matrix's mean square as for single matrices
__global__ __launch_bounds__(64) void batched_pad_kernel(int kind, BatchMatrix *__restrict__ mats,
                                                         int count, const void *data) {
  __shared__ float f[kPadScratch];
  const int i = blockIdx.x;
  if (i >= count) return;
  const BatchMatrix d = mats[i];
  if (d.m <= 0 || d.m >= d.n) return;
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  const double *A = (const double *)data + (size_t)d.offset * C;
  double acc = 0.0;
  for (int e = threadIdx.x; e < d.m * d.n * C; e += 64) {
    const int r = e / (d.n * C), k = e % (d.n * C);
    const double x = A[(size_t)r * d.ld * C + k];
    acc += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  acc = __shfl(acc, 0, 64);  // one value in every lane (the butterfly's order differs by lane)
  const int x = pad_exponent(d.m, d.n, acc, (int)threadIdx.x, 64, f);
  if (threadIdx.x == 0) mats[i].pad_e = x;
}

// per matrix: add its slots in chunk order, normalise, write the typed result
__global__ void batched_finish_kernel(int kind, const BatchMatrix *__restrict__ mats, int count,
                                      const double *__restrict__ slots, perm_out ot, void *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const BatchMatrix d = mats[i];
  if (d.n < 0) return;  // a staged walk writes this matrix's result
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  double rh = 0, rl = 0, ih = 0, il = 0;
  if (d.n == 0) {
    rh = 1.0;
  } else {
    for (uint32_t c = 0; c < d.nchunks; ++c) {
      const double *p = slots + (size_t)(d.first_slot + c) * 2 * C;
      dd_add(rh, rl, p[0], p[1]);
      if (C == 2) dd_add(ih, il, p[2], p[3]);
    }
    const double sc = __builtin_ldexp(1.0, -(d.n - 1));
    rh *= sc; rl *= sc; ih *= sc; il *= sc;
    for (int q = 2; q <= d.n - d.m; ++q) {
      dd_div_d(rh, rl, (double)q);
      if (C == 2) dd_div_d(ih, il, (double)q);
    }
    if (d.pad_e != 0 && d.n > d.m) {
      // padding rows of 2^e: the sum carries 2^(e (n-m)); removed exactly
      const int x = -d.pad_e * (d.n - d.m);
      rh = __builtin_ldexp(rh, x);
      rl = __builtin_ldexp(rl, x);
      ih = __builtin_ldexp(ih, x);
      il = __builtin_ldexp(il, x);
    }
  }
  double h1, l1, h2, l2;
  fast_two_sum(rh, rl, h1, l1);
  fast_two_sum(ih, il, h2, l2);
  double *o = (double *)out;
  switch (ot) {
    case PERM_OUT_F64: o[i] = h1; break;
    case PERM_OUT_DD: o[2 * i] = h1; o[2 * i + 1] = l1; break;
    case PERM_OUT_C128: o[2 * i] = h1; o[2 * i + 1] = h2; break;
    default: o[4 * i] = h1; o[4 * i + 1] = l1; o[4 * i + 2] = h2; o[4 * i + 3] = l2; break;
  }
}

}  // namespace

hipError_t batched_launch_real_a(int n, const BatchBucket &bk, const BatchLaunch &L, hipStream_t s);
hipError_t batched_launch_real_b(int n, const BatchBucket &bk, const BatchLaunch &L, hipStream_t s);
hipError_t batched_launch_cplx_a(int n, const BatchBucket &bk, const BatchLaunch &L, hipStream_t s);
hipError_t batched_launch_cplx_b(int n, const BatchBucket &bk, const BatchLaunch &L, hipStream_t s);
int batched_occ_real_a(int n);
int batched_occ_real_b(int n);
int batched_occ_cplx_a(int n);
int batched_occ_cplx_b(int n);

int batched_blocks_per_cu(int kind, int n) {
  if (kind == ENGINE_CPLX) return n <= 20 ? batched_occ_cplx_a(n) : batched_occ_cplx_b(n);
  return n <= 20 ? batched_occ_real_a(n) : batched_occ_real_b(n);
}

hipError_t launch_batched_bucket(const BatchLaunch &L, int i, hipStream_t s) {
  const BatchBucket &bk = L.buckets[i];
  if (bk.pack > 0)
    return L.kind == ENGINE_CPLX ? launch_batched_small_cplx(bk.n, bk, L, s)
                                 : launch_batched_small_real(bk.n, bk, L, s);
  if (L.kind == ENGINE_CPLX)
    return bk.n <= 20 ? batched_launch_cplx_a(bk.n, bk, L, s) : batched_launch_cplx_b(bk.n, bk, L, s);
  return bk.n <= 20 ? batched_launch_real_a(bk.n, bk, L, s) : batched_launch_real_b(bk.n, bk, L, s);
}

hipError_t launch_batched(const BatchLaunch &L, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (L.scale_pad && L.count > 0) {
    hipLaunchKernelGGL(batched_pad_kernel, dim3(L.count), dim3(64), 0, s, L.kind,
                       L.mats, L.count, L.data);
    e = hipGetLastError();
  }
  for (int i = 0; i < L.nbuckets && e == hipSuccess; ++i) e = launch_batched_bucket(L, i, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_finish_kernel, dim3((L.count + 255) / 256), dim3(256), 0, s, L.kind,
                     L.mats, L.count, L.slots, L.ot, L.out);
  e = hipGetLastError();
  if (e == hipSuccess && L.walk) e = launch_walk_batch(*L.walk, s);
  return e;
}

}  // namespace permgpu
