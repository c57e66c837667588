// Gray-code engine instantiations: int kind, vector lengths 35..40.
#include "internal.h"
#define GRAY_KIND ENGINE_INT
#define GRAY_NV_LO 35
#define GRAY_NV_HI 40
#define GRAY_OCC_NAME gray_occ_int_d
#define GRAY_LAUNCH_NAME gray_launch_int_d
#include "gray_engine.inc"
