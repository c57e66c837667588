// perm_glynn_noalloc: perm_glynn with its device scratch (the Gray walk's
// update table, start vector, per-workgroup partials and padding exponent) in
// a fixed, file-scope device array instead of stream-ordered allocations, for
// callers that cannot allocate (code under graph capture, tight serving
// loops).  The kernels and the plan are those of perm_glynn, so the results
// are bitwise the same.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.h"
#include "runtime.h"

using namespace permgpu;

namespace {

// Largest scratch one call needs: complex n = 48 takes (2*47*48*2 + 96) doubles
// of table and start vector plus 4 doubles per workgroup partial (at most a few
// thousand workgroups on 256 compute units) -- under 150 KiB.
constexpr size_t kNoAllocBytes = PERM_NOALLOC_SCRATCH_BYTES;

// One copy per device, held until the process ends.  In host code `scratch`
// names a host-side stand-in; the device address comes from
// hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
std::vector<void *> g_addr;  // per device; nullptr until looked up

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_address(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PERM_E_HIP;
  std::lock_guard<std::mutex> g(g_mu);
  if ((int)g_addr.size() <= dev) g_addr.resize(dev + 1, nullptr);
  if (!g_addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PERM_E_HIP;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return PERM_OK;
}

}  // namespace

extern "C" int perm_glynn_noalloc(int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                                  perm_out ot, void *dOut, uint32_t flags, void *stream) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  // integer outputs run an overflow pre-check that reads the matrix back
  // through allocated memory
  if (kind == ENGINE_INT) return PERM_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const int tr = m > n;
  const int M = m < n ? m : n, N = m < n ? n : m;
  if (M == 0) return launch_write_one(ot, dOut, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
  if (N > kMaxN) return PERM_E_TOO_LARGE;
  void *buf = nullptr;
  rc = scratch_address(&buf);
  if (rc) return rc;
  return run_gray(0, M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind, -1, 0, buf, kNoAllocBytes);
}
