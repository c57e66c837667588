// Host side of algorithm selection: features, the threshold table and MLP
// inference from loaded weights.  (The network is trained on the GPU by the
// kernels in mlp.hip; this file only evaluates it for single queries.)
#include "selector.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace permgpu {
namespace {

struct Net {
  bool loaded = false;
  float mean[kSelIn] = {0, 0, 0, 0}, stdv[kSelIn] = {1, 1, 1, 1};
  std::vector<float> W1, b1, W2, b2, W3, b3;  // row-major [out][in]
  ThresholdTable table;
  bool has_table = false;
};

std::mutex g_mu;
Net g_net;

}  // namespace

void selector_features(int M, int N, perm_dtype dt, double density, float f[kSelIn]) {
  f[0] = (float)std::log((double)std::max(M, 1));
  f[1] = (float)std::log((double)std::max(N, 1));
  f[2] = (float)(density < 0 ? 1.0 : density);
  f[3] = dt == PERM_C128 ? 1.0f : (dt == PERM_B8 || dt == PERM_I64) ? 2.0f : 0.0f;
}

const ThresholdTable &default_table() {
  // Values fitted to MI355X timings of the three algorithms (square Glynn and
  // Ryser, rectangular Ryser by size) -- see the selector training report.
  static const ThresholdTable t = {{0.0,
                                    /*p1*/ 0.0, /*p2*/ -1.0, /*p3*/ 5.5, /*p4*/ 4.0,
                                    /*p5*/ 1.0, /*p6*/ 0.0, /*p7*/ -0.62, /*p8*/ 8.0}};
  return t;
}

perm_algo table_choice(const ThresholdTable &t, int M, int N) {
  const double r = N > 0 ? (double)M / (double)N : 1.0;
  const double n = (double)N;
  if (n <= t.p[8]) {
    if (M == N && n <= t.p[4]) return PERM_ALGO_COMBINATORIC;
    const double h1 = t.p[1] * r + t.p[2] * n + t.p[3];
    return h1 > 0 ? PERM_ALGO_COMBINATORIC : PERM_ALGO_GLYNN;
  }
  const double h2 = t.p[5] * r + t.p[6] * n + t.p[7];
  return h2 > 0 ? PERM_ALGO_GLYNN : PERM_ALGO_RYSER;
}

static void mlp_forward(const Net &net, const float x[kSelIn], float y[kSelOut]) {
  float z[kSelIn], h1[kSelH], h2[kSelH];
  for (int i = 0; i < kSelIn; ++i) z[i] = (x[i] - net.mean[i]) / net.stdv[i];
  for (int o = 0; o < kSelH; ++o) {
    float s = net.b1[o];
    for (int i = 0; i < kSelIn; ++i) s += net.W1[o * kSelIn + i] * z[i];
    h1[o] = s > 0 ? s : 0;
  }
  for (int o = 0; o < kSelH; ++o) {
    float s = net.b2[o];
    for (int i = 0; i < kSelH; ++i) s += net.W2[o * kSelH + i] * h1[i];
    h2[o] = s > 0 ? s : 0;
  }
  for (int o = 0; o < kSelOut; ++o) {
    float s = net.b3[o];
    for (int i = 0; i < kSelH; ++i) s += net.W3[o * kSelH + i] * h2[i];
    y[o] = s;
  }
}

perm_algo select_algorithm(int M, int N, perm_dtype dt, double density, int *source) {
  std::lock_guard<std::mutex> g(g_mu);
  if (g_net.loaded) {
    float x[kSelIn], y[kSelOut];
    selector_features(M, N, dt, density, x);
    mlp_forward(g_net, x, y);
    int best = 0;
    for (int a = 1; a < kSelOut; ++a)
      if (y[a] < y[best]) best = a;
    if (source) *source = 1;
    return (perm_algo)best;  // output order = perm_algo order
  }
  if (source) *source = 0;
  return table_choice(g_net.has_table ? g_net.table : default_table(), M, N);
}

// Text format (whitespace separated):
//   permgpu-selector 1
//   table p1 p2 p3 p4 p5 p6 p7 p8          (optional)
//   norm mean0..3 std0..3
//   W1 (64x4) b1 (64) W2 (64x64) b2 (64) W3 (3x64) b3 (3)
int selector_load_file(const char *path) {
  std::lock_guard<std::mutex> g(g_mu);
  if (path == nullptr) {
    g_net = Net();
    return PERM_OK;
  }
  FILE *f = std::fopen(path, "r");
  if (!f) return PERM_E_INVALID;
  Net net;
  char tag[64] = {0};
  int ver = 0;
  bool ok = std::fscanf(f, "%63s %d", tag, &ver) == 2 && std::strcmp(tag, "permgpu-selector") == 0;
  auto rd = [&](std::vector<float> &v, size_t n) {
    v.resize(n);
    for (size_t i = 0; i < n && ok; ++i) ok = std::fscanf(f, "%f", &v[i]) == 1;
  };
  while (ok) {
    if (std::fscanf(f, "%63s", tag) != 1) break;
    if (std::strcmp(tag, "table") == 0) {
      for (int i = 1; i <= 8 && ok; ++i) ok = std::fscanf(f, "%lf", &net.table.p[i]) == 1;
      net.has_table = ok;
    } else if (std::strcmp(tag, "norm") == 0) {
      for (int i = 0; i < kSelIn && ok; ++i) ok = std::fscanf(f, "%f", &net.mean[i]) == 1;
      for (int i = 0; i < kSelIn && ok; ++i) ok = std::fscanf(f, "%f", &net.stdv[i]) == 1;
    } else if (std::strcmp(tag, "mlp") == 0) {
      rd(net.W1, kSelH * kSelIn);
      rd(net.b1, kSelH);
      rd(net.W2, kSelH * kSelH);
      rd(net.b2, kSelH);
      rd(net.W3, kSelOut * kSelH);
      rd(net.b3, kSelOut);
      net.loaded = ok;
    } else {
      ok = false;
    }
  }
  std::fclose(f);
  if (!ok) return PERM_E_INVALID;
  for (int i = 0; i < kSelIn; ++i)
    if (!(net.stdv[i] > 0)) net.stdv[i] = 1.0f;
  g_net = net;
  return PERM_OK;
}

}  // namespace permgpu
