// Gray-code engine instantiations: int kind, vector lengths 1..16.
#include "internal.h"
#define GRAY_KIND ENGINE_INT
#define GRAY_NV_LO 1
#define GRAY_NV_HI 16
#define GRAY_OCC_NAME gray_occ_int_a
#define GRAY_LAUNCH_NAME gray_launch_int_a
#include "gray_engine.inc"
