// Algorithm selection for perm_auto: a small MLP over (log m, log n, density,
// dtype) predicting log run time per algorithm, with a threshold table shaped
// like the paper's Alg. 5 (App. B) as the fallback.
#pragma once

#include "../../include/perm.h"

namespace permgpu {

// Network shape: 4 -> 64 -> 64 -> 3, ReLU hidden layers, FP32.
constexpr int kSelIn = 4, kSelH = 64, kSelOut = 3;

// Features of a problem (the order the network sees them).
void selector_features(int M, int N, perm_dtype dt, double density, float f[kSelIn]);

// Threshold table (Alg. 5 structure): with r = m/n,
//   n <= p8:  square and n <= p4 -> combinatoric;
//             else p1 r + p2 n + p3 > 0 -> combinatoric, otherwise Glynn;
//   n >  p8:  p5 r + p6 n + p7 > 0 -> Glynn, otherwise Ryser.
struct ThresholdTable {
  double p[9];  // p[1..8]
};
const ThresholdTable &default_table();
perm_algo table_choice(const ThresholdTable &t, int M, int N);

// The active choice: the loaded network if any, else the table.  *source = 1
// when the network decided.
perm_algo select_algorithm(int M, int N, perm_dtype dt, double density, int *source);

// Load (path != NULL) or unload (NULL) network weights / table values.
int selector_load_file(const char *path);

}  // namespace permgpu
