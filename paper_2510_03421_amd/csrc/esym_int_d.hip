// e_m form of the rectangular permanent: exact integer kind, vector lengths 41..44.
#include "internal.h"
#define ESYM_KIND 2
#define ESYM_NV_LO 41
#define ESYM_NV_HI 44
#define ESYM_OCC_NAME esym_occ_int_d
#define ESYM_LAUNCH_NAME esym_launch_int_d
#include "esym.inc"
