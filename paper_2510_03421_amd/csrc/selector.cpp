// Host side of algorithm selection: features, the threshold table and the
// network's inference from loaded weights for single queries.  (The network
// is trained on the GPU by the kernels in mlp.hip.)
#include "selector.h"

#include <algorithm>
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
  // Alg. 5's structure with values fitted (coordinate search on mean regret)
  // to 4000 timed MI355X cases, m in 2..30, n in m..48, f64 / c128 / 0-1,
  // the e_m rule and the sweep's rank applied after it (rank_algorithms):
  //   n <= 2:  square and n <= 4, or -m/n - n + 5.5 > 0 -> combinatoric, else Glynn;
  //   n >  2:  2 m/n - 0.62 > 0 -> Glynn, else Ryser (by subset size).
  // (With the e_m form taking most rectangular shapes, the definition's
  // small-matrix branch no longer pays off.)
  static const ThresholdTable t = {{0.0,
                                    /*p1*/ -1.0, /*p2*/ -1.0, /*p3*/ 5.5, /*p4*/ 4.0,
                                    /*p5*/ 2.0, /*p6*/ 0.0, /*p7*/ -0.62, /*p8*/ 2.0}};
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

unsigned algo_mask(int M, int N, int kind) {
  unsigned mask = 0;
  // combinatoric: at most 2^40 injective maps
  double maps = 1.0;
  for (int i = 0; i < M; ++i) maps *= (double)(N - i);
  if (maps <= 1099511627776.0) mask |= 1u << PERM_ALGO_COMBINATORIC;
  const int nv_max = kind == 2 ? 40 : 48;  // Gray-walk engine limits (integer / floating)
  if (M == N ? N <= nv_max : (M <= 40 && N <= 64)) mask |= 1u << PERM_ALGO_RYSER;
  if (N <= nv_max) mask |= 1u << PERM_ALGO_GLYNN;
  // the e_m form also runs square matrices (where it is Glynn with the
  // products taken as e_n), and is sometimes the fastest there
  if (M <= N && M <= 32 && N <= 48) mask |= 1u << PERM_ALGO_GLYNN_ESYM;
  if (M <= 28 && N <= 64) mask |= 1u << PERM_ALGO_SWEEP;
  return mask;
}

// log2 of the number of terms each algorithm sums (its cost up to a factor)
double log2_algo_terms(perm_algo a, int M, int N) {
  switch (a) {
    case PERM_ALGO_COMBINATORIC: {
      double l = 0.0;
      for (int i = 0; i < M; ++i) l += std::log2((double)(N - i));
      return l;
    }
    case PERM_ALGO_RYSER: {
      if (M == N) return (double)N;
      double s = 0.0, c = 1.0;  // sum_{k <= M} C(N, k)
      for (int k = 0; k <= M; ++k) {
        s += c;
        c = c * (double)(N - k) / (double)(k + 1);
      }
      return std::log2(s);
    }
    case PERM_ALGO_GLYNN_ESYM: return (double)(M - 1);
    case PERM_ALGO_SWEEP: {
      // states of each size k, times the columns in whose band k lies
      double s = 0.0, c = 1.0;
      for (int k = 0; k <= M; ++k) {
        const int cols = std::min(N - M + 1, std::min(k + 1, N - (M - k)));
        if (cols > 0) s += c * cols;
        c = c * (double)(M - k) / (double)(k + 1);
      }
      return std::log2(std::max(s, 1.0));
    }
    default: return (double)(N - 1);
  }
}

// log2 of a rough operation count: terms times the work of one term
static double log2_algo_ops(perm_algo a, int M, int N) {
  const double t = log2_algo_terms(a, M, N);
  switch (a) {
    case PERM_ALGO_COMBINATORIC: return t + std::log2((double)std::max(M, 1));
    case PERM_ALGO_RYSER: return t + std::log2(2.0 * M);
    case PERM_ALGO_GLYNN: return t + std::log2(2.0 * N);
    case PERM_ALGO_GLYNN_ESYM: return t + std::log2((double)N * (std::min(M, 32) + 1));
    default: return t + std::log2((double)std::max(M, 1));
  }
}

int rank_algorithms(int M, int N, perm_dtype dt, double density, unsigned mask,
                    perm_algo order[kSelOut], int *source) {
  double key[kSelOut];
  int src = 0;
  {
    std::lock_guard<std::mutex> g(g_mu);
    if (g_net.loaded) {
      float x[kSelIn], y[kSelOut];
      selector_features(M, N, dt, density, x);
      mlp_forward(g_net, x, y);
      for (int k = 0; k < kSelOut; ++k) key[k] = y[k];
      src = 1;
    } else {
      const perm_algo c = table_choice(g_net.has_table ? g_net.table : default_table(), M, N);
      for (int k = 0; k < kSelOut; ++k) key[k] = log2_algo_terms(kSelAlgo[k], M, N);
      int first = c;  // output index = perm_algo value for the paper's three
      // the e_m form first when it needs well under the operations of the
      // table's choice (rectangular shapes)
      if ((mask & (1u << PERM_ALGO_GLYNN_ESYM)) &&
          log2_algo_ops(PERM_ALGO_GLYNN_ESYM, M, N) + 1.0 < log2_algo_ops(c, M, N))
        first = 3;
      key[first] = -1e300;
      key[4] = 1e300;  // the sweep last (it trades time for accuracy)
    }
  }
  int idx[kSelOut], cnt = 0;
  for (int k = 0; k < kSelOut; ++k)
    if (mask & (1u << kSelAlgo[k])) idx[cnt++] = k;
  std::stable_sort(idx, idx + cnt, [&](int x, int y) { return key[x] < key[y]; });
  for (int i = 0; i < cnt; ++i) order[i] = kSelAlgo[idx[i]];
  if (source) *source = src;
  return cnt;
}

// Text format (whitespace separated):
//   permgpu-selector 2                     (version 1 files: table only)
//   table p1 p2 p3 p4 p5 p6 p7 p8          (optional)
//   norm mean0..3 std0..3
//   W1 (64x4) b1 (64) W2 (64x64) b2 (64) W3 (5x64) b3 (5)
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
    } else if (std::strcmp(tag, "mlp") == 0 && ver == 2) {  // 5 outputs since version 2
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
