// Staged batch walk kernels (batched_walk.inc): which instantiations exist.
// Each X(kind, esym, nv_lo, nv_hi) entry is one compiled object holding the
// kernels of one engine kind (0 real, 1 complex, 2 exact integer), one term
// kind (0 products: Glynn and Ryser, 1 the e_m form) and the orders
// nv_lo..nv_hi (batches take n <= 32).  The build script reads this list.
#pragma once

#define BATCH_WALK_UNITS(X)                                                        \
  X(0, 0, 1, 32) X(1, 0, 1, 32) X(2, 0, 1, 16) X(2, 0, 17, 32)                     \
  X(0, 1, 1, 32) X(1, 1, 1, 32) X(2, 1, 1, 16) X(2, 1, 17, 24) X(2, 1, 25, 32)
