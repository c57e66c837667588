// Gray-code engine instantiations: int kind, vector lengths 17..26.
#include "internal.h"
#define GRAY_KIND ENGINE_INT
#define GRAY_NV_LO 17
#define GRAY_NV_HI 26
#define GRAY_OCC_NAME gray_occ_int_b
#define GRAY_LAUNCH_NAME gray_launch_int_b
#include "gray_engine.inc"
