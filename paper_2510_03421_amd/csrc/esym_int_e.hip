// e_m form of the rectangular permanent: exact integer kind, vector lengths 45..48.
#include "internal.h"
#define ESYM_KIND 2
#define ESYM_NV_LO 45
#define ESYM_NV_HI 48
#define ESYM_OCC_NAME esym_occ_int_e
#define ESYM_LAUNCH_NAME esym_launch_int_e
#include "esym.inc"
