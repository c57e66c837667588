// C ABI of the selector's training side: timing of the algorithms (the
// training data), the network's GPU primitives (forward, gradient, Adam), the
// training driver that replays one captured epoch, and the weight writer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "mlp.h"
#include "runtime.h"
#include "selector.h"

using namespace permgpu;

namespace {

// Restores normal (untruncated) operation when perm_time returns.
struct TuneGuard {
  explicit TuneGuard(double f) { tune_set(f); }
  ~TuneGuard() { tune_set(1.0); }
};

int run_algo(perm_algo algo, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
             perm_out ot, void *dOut, uint32_t flags, void *stream) {
  switch (algo) {
    case PERM_ALGO_COMBINATORIC:
      return perm_combinatoric(m, n, dt, dA, lda, ot, dOut, flags, stream);
    case PERM_ALGO_RYSER: return perm_ryser(m, n, dt, dA, lda, ot, dOut, flags, stream);
    case PERM_ALGO_GLYNN: return perm_glynn(m, n, dt, dA, lda, ot, dOut, flags, stream);
    case PERM_ALGO_GLYNN_ESYM: return perm_glynn_esym(m, n, dt, dA, lda, ot, dOut, flags, stream);
    case PERM_ALGO_SWEEP: return perm_column_sweep(m, n, dt, dA, lda, ot, dOut, flags, stream);
    default: return PERM_E_INVALID;
  }
}

// splitmix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", 2014): the parameter initialisation's random stream.
uint64_t splitmix64(uint64_t &x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
double uniform01(uint64_t &x) { return (double)(splitmix64(x) >> 11) * 0x1p-53; }

constexpr int NP = kMlpParams, IN = kMlpIn, H = kMlpHidden, OUT = kMlpOut;

// He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero hidden biases,
// output biases at the mean finite target of each output.
void init_params(uint64_t seed, int count, const float *hT, float *P) {
  uint64_t st = seed;
  int o = 0;
  auto fill = [&](int rows, int fan_in) {
    const double a = std::sqrt(6.0 / (double)fan_in);
    for (int i = 0; i < rows * fan_in; ++i) P[o++] = (float)((2.0 * uniform01(st) - 1.0) * a);
  };
  auto zeros = [&](int k) {
    for (int i = 0; i < k; ++i) P[o++] = 0.f;
  };
  fill(H, IN);
  zeros(H);
  fill(H, H);
  zeros(H);
  fill(OUT, H);
  for (int k = 0; k < OUT; ++k) {
    double s = 0.0;
    int c = 0;
    for (int b = 0; b < count; ++b) {
      const float t = hT[(size_t)b * OUT + k];
      if (!std::isnan(t)) {
        s += t;
        ++c;
      }
    }
    P[o++] = c ? (float)(s / c) : 0.f;
  }
}

}  // namespace

extern "C" {

int perm_time(perm_algo algo, int m, int n, perm_dtype dt, const void *dA, int64_t lda,
              perm_out ot, uint32_t flags, double fraction, int reps, void *stream, double *ms,
              double *fraction_run) {
  if (!ms || reps < 1 || !(fraction > 0.0 && fraction <= 1.0)) return PERM_E_INVALID;
  if ((int)algo < 0 || (int)algo > (int)PERM_ALGO_SWEEP || algo == PERM_ALGO_AUTO)
    return PERM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  void *dOut = nullptr;
  if (hipMalloc(&dOut, 64) != hipSuccess) return PERM_E_HIP;
  std::vector<double> t;
  int rc = PERM_OK;
  double ran = 1.0;
  {
    TuneGuard guard(fraction);
    for (int r = 0; r <= reps && rc == PERM_OK; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      rc = run_algo(algo, m, n, dt, dA, lda, ot, dOut, flags, stream);
      if (rc == PERM_OK && hipStreamSynchronize(s) != hipSuccess) rc = PERM_E_HIP;
      const auto t1 = std::chrono::steady_clock::now();
      if (r > 0) t.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
      ran = tune_ran();
    }
  }
  hipFree(dOut);
  if (rc) return rc;
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  if (fraction_run) *fraction_run = ran;
  return PERM_OK;
}

int perm_selector_features(int m, int n, perm_dtype dt, double density, float *x) {
  if (!x || m < 0 || n < 0 || (int)dt < 0 || (int)dt > (int)PERM_B8) return PERM_E_INVALID;
  selector_features(std::min(m, n), std::max(m, n), dt, density, x);
  return PERM_OK;
}

int perm_mlp_forward(const float *dParams, const float *dNorm, const float *dX, int batch,
                     float *dY, void *stream) {
  if (batch < 0 || (batch > 0 && (!dParams || !dNorm || !dX || !dY))) return PERM_E_INVALID;
  return launch_mlp_forward(dParams, dNorm, dX, batch, dY, (hipStream_t)stream) == hipSuccess
             ? PERM_OK
             : PERM_E_HIP;
}

int perm_mlp_grad(const float *dParams, const float *dNorm, const float *dX, const float *dT,
                  int batch, float scale, float *dGrad, float *dLoss, void *stream) {
  if (batch < 0 || !dGrad || !dParams || (batch > 0 && (!dNorm || !dX || !dT)))
    return PERM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const int groups = mlp_groups(batch);
  float *part = nullptr;
  const size_t n = (size_t)groups * (NP + 1) + 1;
  if (hipMallocAsync((void **)&part, sizeof(float) * n, s) != hipSuccess) return PERM_E_HIP;
  hipError_t e = launch_mlp_grad(dParams, dNorm, dX, dT, batch, scale, part,
                                 part + (size_t)groups * NP, dGrad, dLoss, nullptr, nullptr, 0, s);
  hipError_t e2 = hipFreeAsync(part, s);
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

int perm_mlp_adam(float *dParams, const float *dGrad, float *dState, float lr, float beta1,
                  float beta2, float eps, int total_steps, void *stream) {
  if (!dParams || !dGrad || !dState || total_steps < 0) return PERM_E_INVALID;
  return launch_mlp_adam(dParams, dGrad, dState, lr, beta1, beta2, eps, total_steps,
                         (hipStream_t)stream) == hipSuccess
             ? PERM_OK
             : PERM_E_HIP;
}

int perm_selector_train(int count, const float *hX, const float *hT, int epochs, float lr,
                        uint64_t seed, int init, float *hParams, float *hNorm, float *hLoss,
                        void *stream) {
  if (count < 1 || epochs < 1 || !hX || !hT || !hParams || !hNorm || !(lr > 0.f))
    return PERM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  // feature normalisation (mean, standard deviation; 1 for a constant feature)
  for (int f = 0; f < IN; ++f) {
    double mu = 0.0, var = 0.0;
    for (int b = 0; b < count; ++b) mu += hX[(size_t)b * IN + f];
    mu /= count;
    for (int b = 0; b < count; ++b) {
      const double d = hX[(size_t)b * IN + f] - mu;
      var += d * d;
    }
    const double sd = std::sqrt(var / count);
    hNorm[f] = (float)mu;
    hNorm[IN + f] = sd > 1e-6 ? (float)sd : 1.f;
  }
  int finite = 0;
  for (size_t i = 0; i < (size_t)count * OUT; ++i) finite += !std::isnan(hT[i]);
  if (finite == 0) return PERM_E_INVALID;
  if (init) init_params(seed, count, hT, hParams);
  const float scale = 1.f / (float)finite;

  const int groups = mlp_groups(count);
  const size_t nX = (size_t)count * IN, nT = (size_t)count * OUT;
  const size_t nPart = (size_t)groups * NP + groups;
  const size_t total = NP + 8 + nX + nT + nPart + NP + 1 + 3 * NP + (size_t)epochs;
  float *buf = nullptr;
  if (hipMalloc((void **)&buf, sizeof(float) * total) != hipSuccess) return PERM_E_HIP;
  float *dP = buf, *dNorm = dP + NP, *dX = dNorm + 8, *dT = dX + nX, *dPart = dT + nT;
  float *dGrad = dPart + nPart, *dLoss = dGrad + NP, *dState = dLoss + 1,
        *dHist = dState + 3 * NP;
  const int *dStep = (const int *)(dState + 2 * NP);
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipMemcpyAsync(dP, hParams, sizeof(float) * NP, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dNorm, hNorm, sizeof(float) * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dX, hX, sizeof(float) * nX, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dT, hT, sizeof(float) * nT, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(dState, 0, sizeof(float) * 3 * NP, s);
  if (e == hipSuccess) e = hipMemsetAsync(dHist, 0, sizeof(float) * epochs, s);
  // one epoch (gradient, ordered reduction, Adam) captured once, replayed
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t ek = launch_mlp_grad(dP, dNorm, dX, dT, count, scale, dPart,
                                    dPart + (size_t)groups * NP, dGrad, dLoss, dHist, dStep,
                                    epochs, cap);
    if (ek == hipSuccess)
      ek = launch_mlp_adam(dP, dGrad, dState, lr, 0.9f, 0.999f, 1e-8f, epochs, cap);
    e = hipStreamEndCapture(cap, &graph);
    if (ek != hipSuccess) e = ek;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) e = hipGraphLaunch(exec, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hParams, dP, sizeof(float) * NP, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && hLoss)
    e = hipMemcpyAsync(hLoss, dHist, sizeof(float) * epochs, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  if (cap) hipStreamDestroy(cap);
  hipStreamSynchronize(s);
  hipFree(buf);
  return e == hipSuccess ? PERM_OK : PERM_E_HIP;
}

int perm_selector_save(const char *path, const float *hParams, const float *hNorm,
                       const double *hTable) {
  if (!path || !hParams || !hNorm) return PERM_E_INVALID;
  FILE *f = std::fopen(path, "w");
  if (!f) return PERM_E_INVALID;
  std::fprintf(f, "permgpu-selector 2\n");
  if (hTable) {
    std::fprintf(f, "table");
    for (int i = 0; i < 8; ++i) std::fprintf(f, " %.9g", hTable[i]);
    std::fprintf(f, "\n");
  }
  std::fprintf(f, "norm");
  for (int i = 0; i < 8; ++i) std::fprintf(f, " %.9g", hNorm[i]);
  std::fprintf(f, "\nmlp\n");
  for (int i = 0; i < NP; ++i) std::fprintf(f, "%.9g%c", hParams[i], (i % 8 == 7) ? '\n' : ' ');
  std::fprintf(f, "\n");
  const bool ok = std::ferror(f) == 0;
  return (std::fclose(f) == 0 && ok) ? PERM_OK : PERM_E_INVALID;
}

}  // extern "C"
