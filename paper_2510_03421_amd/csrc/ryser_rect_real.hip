// Rectangular Ryser-by-size instantiations, real kind (row counts 1..RECT_MAX_M).
#include "internal.h"
#define RECT_KIND ENGINE_REAL
#define RECT_LAUNCH_NAME launch_ryser_rect_real
#include "ryser_rect.inc"
