// Batched Glynn instantiations: cplx kind, matrix orders 21..32.
#include "internal.h"
#define BATCH_KIND ENGINE_CPLX
#define BATCH_NV_LO 21
#define BATCH_NV_HI 32
#define BATCH_LAUNCH_NAME batched_launch_cplx_b
#define BATCH_OCC_NAME batched_occ_cplx_b
#include "batched.inc"
