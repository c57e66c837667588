// Gray-code engine instantiations: cplx kind, vector lengths 1..24.
#include "internal.h"
#define GRAY_KIND ENGINE_CPLX
#define GRAY_NV_LO 1
#define GRAY_NV_HI 24
#define GRAY_OCC_NAME gray_occ_cplx_a
#define GRAY_LAUNCH_NAME gray_launch_cplx_a
#include "gray_engine.inc"
