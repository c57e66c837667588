// Gray-code engine instantiations: cplx kind, vector lengths 41..48.
#include "internal.h"
#define GRAY_KIND ENGINE_CPLX
#define GRAY_NV_LO 41
#define GRAY_NV_HI 48
#define GRAY_OCC_NAME gray_occ_cplx_c
#define GRAY_LAUNCH_NAME gray_launch_cplx_c
#include "gray_engine.inc"
