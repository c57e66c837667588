// Banded e_m kernels (esym_band.inc): which (kind, m) ranges exist.  Each
// X(kind, m_lo, m_hi) entry is one compiled object holding the kernels for
// m_lo <= m <= m_hi and m <= n <= ESYM_BAND_MAX_N (kind 0 real, 1 complex).
// Smaller m (at most 2^12 terms, a launch-latency-bound walk) and the
// exact-integer kind use the generic kernels of esym.inc.  The build script
// reads this list to compile the objects.
#pragma once

#define ESYM_BAND_MIN_M 14
#define ESYM_BAND_MAX_N 48
#define ESYM_BAND_RANGES(X)                                                          \
  X(0, 14, 15) X(0, 16, 17) X(0, 18, 19) X(0, 20, 21) X(0, 22, 23) X(0, 24, 25)     \
  X(0, 26, 28) X(0, 29, 32)                                                          \
  X(1, 14, 15) X(1, 16, 17) X(1, 18, 19) X(1, 20, 21) X(1, 22, 23) X(1, 24, 25)     \
  X(1, 26, 28) X(1, 29, 32)
