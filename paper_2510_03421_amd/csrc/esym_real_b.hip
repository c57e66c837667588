// e_m form of the rectangular permanent: real kind, vector lengths 25..48.
#include "internal.h"
#define ESYM_KIND 0
#define ESYM_NV_LO 25
#define ESYM_NV_HI 48
#define ESYM_OCC_NAME esym_occ_real_b
#define ESYM_LAUNCH_NAME esym_launch_real_b
#include "esym.inc"
