// e_m form of the rectangular permanent: exact integer kind, vector lengths 33..40.
#include "internal.h"
#define ESYM_KIND 2
#define ESYM_NV_LO 33
#define ESYM_NV_HI 40
#define ESYM_OCC_NAME esym_occ_int_c
#define ESYM_LAUNCH_NAME esym_launch_int_c
#include "esym.inc"
