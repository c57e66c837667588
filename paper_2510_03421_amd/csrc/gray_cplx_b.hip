// Gray-code engine instantiations: cplx kind, vector lengths 25..40.
#include "internal.h"
#define GRAY_KIND ENGINE_CPLX
#define GRAY_NV_LO 25
#define GRAY_NV_HI 40
#define GRAY_OCC_NAME gray_occ_cplx_b
#define GRAY_LAUNCH_NAME gray_launch_cplx_b
#include "gray_engine.inc"
