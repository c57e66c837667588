// Batched Glynn instantiations: real kind, matrix orders 1..20.
#include "internal.h"
#define BATCH_KIND ENGINE_REAL
#define BATCH_NV_LO 1
#define BATCH_NV_HI 20
#define BATCH_LAUNCH_NAME batched_launch_real_a
#define BATCH_OCC_NAME batched_occ_real_a
#include "batched.inc"
