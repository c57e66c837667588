// Internal declarations of the selector network's kernels (mlp.hip) and of
// its host-side training driver.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace permgpu {

constexpr int kMlpIn = 4, kMlpHidden = 64, kMlpOut = 5;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpOut * kMlpHidden + kMlpOut;  // 4805

// Number of per-workgroup partial gradients the gradient kernel writes for a
// batch (part_grad holds mlp_groups(batch) * kMlpParams floats, part_loss
// mlp_groups(batch) floats).
int mlp_groups(int batch);

hipError_t launch_mlp_forward(const float *P, const float *norm, const float *X, int batch,
                              float *Y, hipStream_t s);
// Gradient kernel + ordered reduction into grad (and the loss into *loss,
// and history[*step] when history and step are given).
hipError_t launch_mlp_grad(const float *P, const float *norm, const float *X, const float *T,
                           int batch, float scale, float *part_grad, float *part_loss, float *grad,
                           float *loss, float *history, const int *step, int hist_len,
                           hipStream_t s);
// state = m[kMlpParams] | v[kMlpParams] | int32 step count[kMlpParams]
hipError_t launch_mlp_adam(float *P, const float *grad, float *state, float lr, float beta1,
                           float beta2, float eps, int total_steps, hipStream_t s);

}  // namespace permgpu
