// Gray-code engine instantiations: int kind, vector lengths 27..34.
#include "internal.h"
#define GRAY_KIND ENGINE_INT
#define GRAY_NV_LO 27
#define GRAY_NV_HI 34
#define GRAY_OCC_NAME gray_occ_int_c
#define GRAY_LAUNCH_NAME gray_launch_int_c
#include "gray_engine.inc"
