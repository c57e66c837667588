// Rectangular Ryser-by-size instantiations, cplx kind (row counts 1..RECT_MAX_M).
#include "internal.h"
#define RECT_KIND ENGINE_CPLX
#define RECT_LAUNCH_NAME launch_ryser_rect_cplx
#include "ryser_rect.inc"
