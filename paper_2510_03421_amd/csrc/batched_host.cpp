// C ABI of the batched path (plan, run, destroy).
#include <hip/hip_runtime.h>

#include "runtime.h"

extern "C" {

int perm_batch_plan_create(int count, const int32_t *hM, const int32_t *hN,
                           const int64_t *hOffset, const int64_t *hLd, perm_dtype dt,
                           perm_out ot, perm_algo algo, uint32_t flags, perm_batch_plan **plan) {
  (void)count; (void)hM; (void)hN; (void)hOffset; (void)hLd; (void)dt; (void)ot; (void)algo;
  (void)flags;
  if (plan) *plan = nullptr;
  return PERM_E_UNSUPPORTED;
}

int perm_batch_plan_run(perm_batch_plan *plan, const void *dData, void *dOut, void *stream) {
  (void)plan; (void)dData; (void)dOut; (void)stream;
  return PERM_E_UNSUPPORTED;
}

int perm_batch_plan_destroy(perm_batch_plan *plan) {
  (void)plan;
  return PERM_OK;
}

int perm_glynn_batched(int count, const int32_t *hM, const int32_t *hN, const int64_t *hOffset,
                       const int64_t *hLd, perm_dtype dt, const void *dData, perm_out ot,
                       void *dOut, uint32_t flags, void *stream) {
  (void)count; (void)hM; (void)hN; (void)hOffset; (void)hLd; (void)dt; (void)dData; (void)ot;
  (void)dOut; (void)flags; (void)stream;
  return PERM_E_UNSUPPORTED;
}

}  // extern "C"
