// Batched Glynn, several matrices per wave: complex kind, orders 1..BATCH_PACK_MAX_N.
#include "internal.h"
#define BATCH_KIND ENGINE_CPLX
#define BATCH_SMALL_LAUNCH_NAME launch_batched_small_cplx
#include "batched_small.inc"
