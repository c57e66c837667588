// Rectangular Ryser-by-size instantiations, int kind (row counts 1..RECT_MAX_M).
#include "internal.h"
#define RECT_KIND ENGINE_INT
#define RECT_LAUNCH_NAME launch_ryser_rect_int
#include "ryser_rect.inc"
