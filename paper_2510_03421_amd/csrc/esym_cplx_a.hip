// e_m form of the rectangular permanent: complex kind, vector lengths 1..24.
#include "internal.h"
#define ESYM_KIND 1
#define ESYM_NV_LO 1
#define ESYM_NV_HI 24
#define ESYM_OCC_NAME esym_occ_cplx_a
#define ESYM_LAUNCH_NAME esym_launch_cplx_a
#include "esym.inc"
