// e_m form of the rectangular permanent: real kind, vector lengths 1..24.
#include "internal.h"
#define ESYM_KIND 0
#define ESYM_NV_LO 1
#define ESYM_NV_HI 24
#define ESYM_OCC_NAME esym_occ_real_a
#define ESYM_LAUNCH_NAME esym_launch_real_a
#include "esym.inc"
