// e_m form of the rectangular permanent: exact integer kind, vector lengths 1..24.
#include "internal.h"
#define ESYM_KIND 2
#define ESYM_NV_LO 1
#define ESYM_NV_HI 24
#define ESYM_OCC_NAME esym_occ_int_a
#define ESYM_LAUNCH_NAME esym_launch_int_a
#include "esym.inc"
