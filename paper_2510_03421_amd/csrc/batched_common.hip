// Batched Glynn: per-matrix finishing kernel and the launch sequence (one
// kernel per matrix order -- packed small orders or chunked persistent ones --
// then the finish).
#include "device_common.h"
#include "internal.h"

namespace permgpu {
namespace {

// per matrix: add its slots in chunk order, normalise, write the typed result
__global__ void batched_finish_kernel(int kind, const BatchMatrix *__restrict__ mats, int count,
                                      const double *__restrict__ slots, perm_out ot, void *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const BatchMatrix d = mats[i];
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
  for (int i = 0; i < L.nbuckets && e == hipSuccess; ++i) e = launch_batched_bucket(L, i, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_finish_kernel, dim3((L.count + 255) / 256), dim3(256), 0, s, L.kind,
                     L.mats, L.count, L.slots, L.ot, L.out);
  return hipGetLastError();
}

}  // namespace permgpu
