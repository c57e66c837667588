// Gray-code engine instantiations: real kind, paired walk (two blocks per
// lane at a time), vector lengths GRAY_PAIR_MIN_NV..GRAY_PAIR_MAX_NV.
#include "internal.h"
#define GRAY_KIND ENGINE_REAL
#define GRAY_PAIR 1
#define GRAY_NV_LO GRAY_PAIR_MIN_NV
#define GRAY_NV_HI GRAY_PAIR_MAX_NV
#define GRAY_OCC_NAME gray_occ_real_pair
#define GRAY_LAUNCH_NAME gray_launch_real_pair
#include "gray_engine.inc"
