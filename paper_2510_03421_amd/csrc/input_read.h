// Reading one logical entry of the caller's matrix on the device.
#pragma once
#include "internal.h"

namespace permgpu {

// Logical entry (i, j) of A (m <= n after orientation; tr reads A^T in
// place) as (re, im): int64 converted to binary64 (exact below 2^53), a 0/1
// byte as 0 or 1 (any nonzero byte reads as 1).
__device__ __forceinline__ void read_entry(perm_dtype dt, const void *dA, int64_t lda, int tr,
                                           int i, int j, double &re, double &im) {
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
}

}  // namespace permgpu
