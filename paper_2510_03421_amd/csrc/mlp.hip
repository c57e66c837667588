// The algorithm selector's network on the GPU: forward pass, gradient of the
// masked squared error on log run times, and Adam, all in FP32.
//
// Network 4 -> 64 -> 64 -> 3 with ReLU hidden layers on normalised features
// z = (x - mean) / std.  Parameters are one flat array:
//   W1[64][4] | b1[64] | W2[64][64] | b2[64] | W3[5][64] | b3[5]   (4805 floats)
// Targets t[b][k] are log run times; a NaN target (algorithm not available
// for that shape) takes no part in the loss
//   L = scale * sum_{b,k: t finite} (y[b][k] - t[b][k])^2.
//
// The gradient is deterministic: each workgroup handles kSamples consecutive
// samples and writes one partial gradient; a second kernel adds the partials
// in workgroup order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mlp.h"

namespace permgpu {
namespace {

constexpr int IN = kMlpIn, H = kMlpHidden, OUT = kMlpOut;
constexpr int OW1 = 0, OB1 = OW1 + H * IN, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
              OB3 = OW3 + OUT * H, NP = OB3 + OUT;
static_assert(NP == kMlpParams, "parameter layout");

constexpr int kThreads = 256;
constexpr int kSamples = 16;  // samples per workgroup in the gradient kernel

// ---- forward only: one thread per sample, activations in registers ----
__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(const float *__restrict__ P,
                                                               const float *__restrict__ norm,
                                                               const float *__restrict__ X,
                                                               int batch, float *__restrict__ Y) {
  __shared__ float sp[NP];
  for (int i = threadIdx.x; i < NP; i += blockDim.x) sp[i] = P[i];
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  float z[IN];
#pragma unroll
  for (int i = 0; i < IN; ++i) z[i] = (X[(size_t)b * IN + i] - norm[i]) / norm[IN + i];
  float h1[H];
#pragma unroll
  for (int o = 0; o < H; ++o) {
    float s = sp[OB1 + o];
#pragma unroll
    for (int i = 0; i < IN; ++i) s = fmaf(sp[OW1 + o * IN + i], z[i], s);
    h1[o] = fmaxf(s, 0.f);
  }
  float y[OUT];
#pragma unroll
  for (int k = 0; k < OUT; ++k) y[k] = sp[OB3 + k];
  for (int o = 0; o < H; ++o) {
    float s = sp[OB2 + o];
#pragma unroll
    for (int i = 0; i < H; ++i) s = fmaf(sp[OW2 + o * H + i], h1[i], s);
    const float h2 = fmaxf(s, 0.f);
#pragma unroll
    for (int k = 0; k < OUT; ++k) y[k] = fmaf(sp[OW3 + k * H + o], h2, y[k]);
  }
#pragma unroll
  for (int k = 0; k < OUT; ++k) Y[(size_t)b * OUT + k] = y[k];
}

// ---- gradient: forward + backward for kSamples samples per workgroup, then
// that workgroup's share of every parameter's gradient ----
__global__ __launch_bounds__(kThreads) void mlp_grad_kernel(
    const float *__restrict__ P, const float *__restrict__ norm, const float *__restrict__ X,
    const float *__restrict__ T, int batch, float scale, float *__restrict__ part_grad,
    float *__restrict__ part_loss) {
  __shared__ float sp[NP];
  __shared__ float w2t[H * H];  // W2 transposed: w2t[i][o] = W2[o][i]
  __shared__ float zs[kSamples][IN];
  __shared__ float h1s[kSamples][H], h2s[kSamples][H];
  __shared__ float d1s[kSamples][H], d2s[kSamples][H];
  __shared__ float dys[kSamples][OUT];
  __shared__ float ls[kSamples];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * kSamples;
  for (int i = tid; i < NP; i += kThreads) sp[i] = P[i];
  for (int i = tid; i < H * H; i += kThreads) w2t[(i % H) * H + i / H] = P[OW2 + i];
  for (int i = tid; i < kSamples * IN; i += kThreads) {
    const int s = i / IN, f = i % IN;
    const int b = s0 + s;
    zs[s][f] = b < batch ? (X[(size_t)b * IN + f] - norm[f]) / norm[IN + f] : 0.f;
  }
  __syncthreads();
  // layer 1
  for (int i = tid; i < kSamples * H; i += kThreads) {
    const int s = i / H, o = i % H;
    float a = sp[OB1 + o];
#pragma unroll
    for (int f = 0; f < IN; ++f) a = fmaf(sp[OW1 + o * IN + f], zs[s][f], a);
    h1s[s][o] = fmaxf(a, 0.f);
  }
  __syncthreads();
  // layer 2 (lanes over o read consecutive entries of W2^T)
  for (int i = tid; i < kSamples * H; i += kThreads) {
    const int s = i / H, o = i % H;
    float a = sp[OB2 + o];
#pragma unroll 8
    for (int j = 0; j < H; ++j) a = fmaf(w2t[j * H + o], h1s[s][j], a);
    h2s[s][o] = fmaxf(a, 0.f);
  }
  __syncthreads();
  // output, loss and dL/dy
  if (tid < kSamples) {
    const int s = tid, b = s0 + s;
    float l = 0.f;
#pragma unroll
    for (int k = 0; k < OUT; ++k) {
      float y = sp[OB3 + k];
      for (int j = 0; j < H; ++j) y = fmaf(sp[OW3 + k * H + j], h2s[s][j], y);
      float d = 0.f;
      if (b < batch) {
        const float t = T[(size_t)b * OUT + k];
        if (!isnan(t)) {
          const float e = y - t;
          l = fmaf(e, e, l);
          d = 2.f * scale * e;
        }
      }
      dys[s][k] = d;
    }
    ls[s] = l;
  }
  __syncthreads();
  // back through layer 3 and the second ReLU
  for (int i = tid; i < kSamples * H; i += kThreads) {
    const int s = i / H, o = i % H;
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < OUT; ++k) a = fmaf(sp[OW3 + k * H + o], dys[s][k], a);
    d2s[s][o] = h2s[s][o] > 0.f ? a : 0.f;
  }
  __syncthreads();
  // back through layer 2 and the first ReLU (lanes over j read rows of W2)
  for (int i = tid; i < kSamples * H; i += kThreads) {
    const int s = i / H, j = i % H;
    float a = 0.f;
#pragma unroll 8
    for (int o = 0; o < H; ++o) a = fmaf(sp[OW2 + o * H + j], d2s[s][o], a);
    d1s[s][j] = h1s[s][j] > 0.f ? a : 0.f;
  }
  __syncthreads();
  // this workgroup's gradient share, samples in order
  float *g = part_grad + (size_t)blockIdx.x * NP;
  for (int p = tid; p < NP; p += kThreads) {
    float a = 0.f;
    if (p < OB1) {
      const int o = p / IN, f = p % IN;
      for (int s = 0; s < kSamples; ++s) a = fmaf(d1s[s][o], zs[s][f], a);
    } else if (p < OW2) {
      const int o = p - OB1;
      for (int s = 0; s < kSamples; ++s) a += d1s[s][o];
    } else if (p < OB2) {
      const int o = (p - OW2) / H, j = (p - OW2) % H;
      for (int s = 0; s < kSamples; ++s) a = fmaf(d2s[s][o], h1s[s][j], a);
    } else if (p < OW3) {
      const int o = p - OB2;
      for (int s = 0; s < kSamples; ++s) a += d2s[s][o];
    } else if (p < OB3) {
      const int k = (p - OW3) / H, j = (p - OW3) % H;
      for (int s = 0; s < kSamples; ++s) a = fmaf(dys[s][k], h2s[s][j], a);
    } else {
      const int k = p - OB3;
      for (int s = 0; s < kSamples; ++s) a += dys[s][k];
    }
    g[p] = a;
  }
  if (tid == 0) {
    float l = 0.f;
    for (int s = 0; s < kSamples; ++s) l += ls[s];
    part_loss[blockIdx.x] = l * scale;
  }
}

// Sum of the per-workgroup partials in workgroup order.  The loss goes to
// loss[0], and also to history[*step] when history is given and the step
// counter (the Adam step count of parameter 0) is below hist_len.
__global__ __launch_bounds__(kThreads) void mlp_reduce_kernel(
    const float *__restrict__ part_grad, const float *__restrict__ part_loss, int groups,
    float *__restrict__ grad, float *__restrict__ loss, float *__restrict__ history,
    const int *__restrict__ step, int hist_len) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    float a = 0.f;
    for (int g = 0; g < groups; ++g) a += part_grad[(size_t)g * NP + p];
    grad[p] = a;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float l = 0.f;
    for (int g = 0; g < groups; ++g) l += part_loss[g];
    if (loss) loss[0] = l;
    if (history && step) {
      const int e = step[0];
      if (e >= 0 && e < hist_len) history[e] = l;
    }
  }
}

// Adam with bias correction; each parameter keeps its own step count, so a
// captured epoch can be replayed without changing kernel arguments.  With
// total_steps > 0 the learning rate follows a cosine decay to 0 over
// total_steps.
__global__ __launch_bounds__(kThreads) void mlp_adam_kernel(float *__restrict__ P,
                                                            const float *__restrict__ grad,
                                                            float *__restrict__ state, float lr,
                                                            float beta1, float beta2, float eps,
                                                            int total_steps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  float *m = state;
  float *v = state + NP;
  int *steps = (int *)(state + 2 * NP);
  const int t = steps[p] + 1;
  steps[p] = t;
  const float g = grad[p];
  const float mt = beta1 * m[p] + (1.f - beta1) * g;
  const float vt = beta2 * v[p] + (1.f - beta2) * g * g;
  m[p] = mt;
  v[p] = vt;
  const float mhat = mt / (1.f - powf(beta1, (float)t));
  const float vhat = vt / (1.f - powf(beta2, (float)t));
  float rate = lr;
  if (total_steps > 0) {
    const float x = fminf((float)t, (float)total_steps) / (float)total_steps;
    rate = lr * 0.5f * (1.f + cosf(3.14159265358979f * x));
  }
  P[p] -= rate * mhat / (sqrtf(vhat) + eps);
}

}  // namespace

int mlp_groups(int batch) { return (batch + kSamples - 1) / kSamples; }

hipError_t launch_mlp_forward(const float *P, const float *norm, const float *X, int batch,
                              float *Y, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const int grid = (batch + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(kThreads), 0, s, P, norm, X, batch, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *P, const float *norm, const float *X, const float *T,
                           int batch, float scale, float *part_grad, float *part_loss, float *grad,
                           float *loss, float *history, const int *step, int hist_len,
                           hipStream_t s) {
  const int groups = mlp_groups(batch);
  if (groups > 0) {
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(groups), dim3(kThreads), 0, s, P, norm, X, T, batch,
                       scale, part_grad, part_loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((NP + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     part_grad, part_loss, groups, grad, loss, history, step, hist_len);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float *P, const float *grad, float *state, float lr, float beta1,
                           float beta2, float eps, int total_steps, hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((NP + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     P, grad, state, lr, beta1, beta2, eps, total_steps);
  return hipGetLastError();
}

}  // namespace permgpu
