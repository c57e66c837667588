// Algorithm selection for perm_auto: a small MLP over (log m, log n, density,
// dtype) predicting log run time per algorithm, with a threshold table shaped
// like the paper's Alg. 5 (App. B) as the fallback.
#pragma once

#include "../../include/perm.h"
#include "mlp.h"

namespace permgpu {

// Network shape: 4 -> 64 -> 64 -> 5, ReLU hidden layers, FP32 (the same
// network the GPU kernels train).  Output k predicts the log run time of
// kSelAlgo[k].
constexpr int kSelIn = kMlpIn, kSelH = kMlpHidden, kSelOut = kMlpOut;
constexpr perm_algo kSelAlgo[kSelOut] = {PERM_ALGO_COMBINATORIC, PERM_ALGO_RYSER, PERM_ALGO_GLYNN,
                                         PERM_ALGO_GLYNN_ESYM, PERM_ALGO_SWEEP};

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

// log2 of the number of terms algorithm a sums on the logical M x N shape:
// injective maps, column subsets (square 2^N, by size sum_{s<=M} C(N, s)),
// Glynn's 2^(N-1) sign vectors, the e_m form's 2^(M-1), or the column
// sweep's state updates.
double log2_algo_terms(perm_algo a, int M, int N);

// Algorithms whose size limits admit the logical M x N shape (M <= N) for an
// engine kind: bit a set <=> perm_algo a can run it (the e_m form only for
// M < N).
unsigned algo_mask(int M, int N, int kind);

// The algorithms of `mask` in the order perm_auto tries them: by the loaded
// network's predicted log time if a network is loaded (*source = 1); else
// (*source = 0) the table's choice among the paper's three algorithms first
// -- or the e_m form, for M < N, when its operation count is below half of
// that choice's -- and the rest by their term counts.  Returns how many
// entries of order[] were filled.
int rank_algorithms(int M, int N, perm_dtype dt, double density, unsigned mask,
                    perm_algo order[kSelOut], int *source);

// Load (path != NULL) or unload (NULL) network weights / table values.
int selector_load_file(const char *path);

}  // namespace permgpu
