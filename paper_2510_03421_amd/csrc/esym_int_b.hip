// e_m form of the rectangular permanent: exact integer kind, vector lengths 25..32.
#include "internal.h"
#define ESYM_KIND 2
#define ESYM_NV_LO 25
#define ESYM_NV_HI 32
#define ESYM_OCC_NAME esym_occ_int_b
#define ESYM_LAUNCH_NAME esym_launch_int_b
#include "esym.inc"
