// C ABI: the combinatoric path, algorithm selection (perm_auto / perm_select)
// and the selector weight loader.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.h"
#include "selector.h"

using namespace permgpu;

namespace permgpu {

int run_combinatoric(int M, int N, perm_dtype dt, const void *dA, int64_t lda, int tr,
                     perm_out ot, void *dOut, uint32_t flags, hipStream_t s, int kind) {
  // number of injective maps N!/(N-M)!, limited to 2^40
  u128_host total = 1;
  for (int i = 0; i < M; ++i) {
    total *= (u128_host)(N - i);
    if (total > ((u128_host)1 << 40)) return PERM_E_TOO_LARGE;
  }
  if (kind == ENGINE_INT) {
    int pl = 0;
    int rc = int_precheck(1, M, N, dt, dA, lda, tr, ot, flags, s, pl);
    if (rc == PERM_E_OVERFLOW && (flags & PERM_FLAG_WRAP)) rc = PERM_OK;  // exact mod 2^128
    if (rc) return rc;
  }
  const int cus = device_cus();
  const int bpc = combinatoric_blocks_per_cu(kind, M, N);
  if (cus <= 0 || bpc <= 0) return PERM_E_HIP;
  // prefix length q: the shortest whose prefix count gives every resident lane
  // at least four prefixes (all rows when the maps fit the lanes); rounds of
  // T lanes, T the smallest multiple of 256 covering the prefixes in that
  // many rounds
  const uint64_t lanes_max = (uint64_t)cus * (uint64_t)bpc * 256u;
  CombPlan c;
  c.q = M;
  if ((uint64_t)total > lanes_max) {
    u128_host p = 1;
    for (int q = 0; q <= M; ++q) {
      if (q > 0) p *= (u128_host)(N - q + 1);
      if (p >= (u128_host)4 * lanes_max) {
        c.q = q;
        break;
      }
    }
  }
  u128_host prefixes = 1;
  for (int i = 0; i < c.q; ++i) prefixes *= (u128_host)(N - i);
  c.prefixes = (uint64_t)prefixes;
  c.suffixes = (uint64_t)(total / prefixes);
  const uint64_t rounds = (c.prefixes + lanes_max - 1) / lanes_max;
  const uint64_t T = ((c.prefixes + rounds - 1) / rounds + 255) / 256 * 256;
  c.grid = (int)(T / 256);
  c.rounds = (uint32_t)rounds;
  const double f = tune_fraction();
  if (f < 1.0) {
    // whole rounds of prefixes, at least one
    c.rounds = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(rounds, (uint64_t)std::llround((double)rounds * f)));
  }
  const uint64_t ran = std::min<uint64_t>(c.prefixes, (uint64_t)c.rounds * T) * c.suffixes;
  tune_record((double)ran / (double)(uint64_t)total);
  const int grid = c.grid;
  const int C = kind == ENGINE_CPLX ? 2 : 1;
  double *part = nullptr;
  if (hipMallocAsync((void **)&part, sizeof(double) * 2 * C * (size_t)grid, s) != hipSuccess)
    return PERM_E_HIP;
  profile_begin(s);
  hipError_t e = launch_combinatoric(kind, M, N, dt, dA, lda, tr, c, part, s);
  profile_end(s);
  if (e == hipSuccess) {
    Finish f;
    f.mode = FINISH_PLAIN;
    f.m = M;
    f.n = N;
    f.ot = ot;
    e = launch_finish(kind, part, grid, f, dOut, s);
  }
  hipError_t e2 = hipFreeAsync(part, s);
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

}  // namespace permgpu

extern "C" {

int perm_combinatoric(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot,
                      void *dOut, uint32_t flags, void *stream) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int tr = m > n;
  const int M = std::min(m, n), N = std::max(m, n);
  if (M == 0) return launch_write_one(ot, dOut, s) == hipSuccess ? PERM_OK : PERM_E_HIP;
  if (N > kMaxN) return PERM_E_TOO_LARGE;
  return run_combinatoric(M, N, dt, dA, lda, tr, ot, dOut, flags, s, kind);
}

int perm_select(int m, int n, perm_dtype dt, double density, perm_algo *chosen, int *source) {
  if (m < 0 || n < 0 || (int)dt < 0 || (int)dt > (int)PERM_B8) return PERM_E_INVALID;
  const int M = std::min(m, n), N = std::max(m, n);
  // the engine kind of the default output type of dt (integers: exact)
  const int kind = dt == PERM_C128 ? ENGINE_CPLX : dt == PERM_F64 ? ENGINE_REAL : ENGINE_INT;
  perm_algo order[kSelOut];
  int src = 0;
  const int cnt = rank_algorithms(M, N, dt, density, algo_mask(M, N, kind), order, &src);
  if (cnt == 0) return PERM_E_TOO_LARGE;
  if (chosen) *chosen = order[0];
  if (source) *source = src;
  return PERM_OK;
}

static int run_one(perm_algo a, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
                   perm_out ot, void *dOut, uint32_t flags, void *stream) {
  switch (a) {
    case PERM_ALGO_COMBINATORIC: return perm_combinatoric(m, n, dt, dA, lda, ot, dOut, flags, stream);
    case PERM_ALGO_RYSER: return perm_ryser(m, n, dt, dA, lda, ot, dOut, flags, stream);
    case PERM_ALGO_GLYNN_ESYM: return perm_glynn_esym(m, n, dt, dA, lda, ot, dOut, flags, stream);
    case PERM_ALGO_SWEEP: return perm_column_sweep(m, n, dt, dA, lda, ot, dOut, flags, stream);
    default: return perm_glynn(m, n, dt, dA, lda, ot, dOut, flags, stream);
  }
}

int perm_auto(int m, int n, perm_dtype dt, const void *dA, int64_t lda, perm_out ot, void *dOut,
              uint32_t flags, void *stream, double density, perm_algo *chosen) {
  int kind = 0;
  int rc = validate(m, n, dt, dA, lda, ot, dOut, kind);
  if (rc) return rc;
  const int M = std::min(m, n), N = std::max(m, n);
  perm_algo order[kSelOut];
  int src = 0;
  const int cnt = rank_algorithms(M, N, dt, density, algo_mask(M, N, kind), order, &src);
  if (cnt == 0) return PERM_E_TOO_LARGE;
  // in ranked order; an algorithm that refuses the input (size limit, or an
  // integer bound that only it cannot meet, such as Glynn's extra factor
  // 2^(n-1) (n-m)!) passes to the next one
  rc = PERM_E_TOO_LARGE;
  for (int i = 0; i < cnt; ++i) {
    rc = run_one(order[i], m, n, dt, dA, lda, ot, dOut, flags, stream);
    if (rc != PERM_E_TOO_LARGE && rc != PERM_E_OVERFLOW) {
      if (rc == PERM_OK && chosen) *chosen = order[i];
      return rc;
    }
  }
  return rc;
}

int perm_selector_load(const char *path) { return selector_load_file(path); }

}  // extern "C"
