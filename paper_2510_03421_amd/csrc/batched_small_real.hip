// Batched Glynn, several matrices per wave: real kind, orders 1..BATCH_PACK_MAX_N.
#include "internal.h"
#define BATCH_KIND ENGINE_REAL
#define BATCH_SMALL_LAUNCH_NAME launch_batched_small_real
#include "batched_small.inc"
