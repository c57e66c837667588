// The padding value 2^e of the floating-point rectangular Glynn sum (Sec. 1.2
// Eq. glynn_filled_matrix pads an m x n matrix with n - m rows; any nonzero
// constant c gives the same permanent after dividing by c^(n-m)).
//
// The value decides how much the sum cancels.  A term is prod_j (x_j + c P):
// x_j the data rows' signed column sum (variance s2 = m mean|a_ij|^2 over
// random signs), P the sum of the n - m padding signs, which takes the value
// k - 2t (k = n - m) for C(k, t) sign vectors.  The sum's value carries the
// factor c^k, its terms' magnitudes about sqrt(s2 + c^2 P^2)^n, so the
// relative rounding error grows with
//   F(c) = ln sum_t C(k, t) (s2 + c^2 (k - 2t)^2)^(n/2) - k ln c:
// steeply for c too small (the padding's share is lost, a power k of c),
// mildly for c too large (a power m).  e minimises F over 21 candidates
// around the balance point sqrt(s2 / k).  (Measured on uniform real and
// Gaussian complex inputs: within one step of the best power of two.)
#pragma once
#include "internal.h"

namespace permgpu {

constexpr int kPadCandidates = 21;
constexpr int kPadMaxK = 48;  // n - m < 48 (n <= 48 where Glynn pads)
// workgroup shared scratch of pad_exponent: the terms of every (candidate, t)
// pair, the log binomials and the candidates' values
constexpr int kPadScratch = kPadCandidates * kPadMaxK + kPadMaxK + kPadCandidates;

// Called by every one of the `nt` threads of a workgroup (tid = thread
// index) with the sum of |a_ij|^2 over the m x n entries; `f` is workgroup
// shared scratch of kPadScratch floats.  Returns e in every thread.
__device__ inline int pad_exponent(int m, int n, double sum_sq, int tid, int nt, float *f) {
  const int k = n - m;
  if (k <= 0 || k >= kPadMaxK || !(sum_sq > 0.0)) return 0;
  float *val = f, *lnc = f + kPadCandidates * kPadMaxK, *F = lnc + kPadMaxK;
  const float s2 = (float)(sum_sq / (double)n);
  const int e_mid = (int)rintf(0.5f * log2f(s2 / (float)k));
  const int e_lo = e_mid - kPadCandidates / 2;
  const int T = k + 1;  // padding sums P = k - 2t, t = 0..k
  for (int t = tid; t < T; t += nt)
    lnc[t] = lgammaf((float)k + 1.0f) - lgammaf((float)t + 1.0f) - lgammaf((float)(k - t) + 1.0f);
  __syncthreads();
  for (int idx = tid; idx < kPadCandidates * T; idx += nt) {
    const int ci = idx / T, t = idx % T;
    const float P = (float)(k - 2 * t);
    const float c2 = exp2f(2.0f * (float)(e_lo + ci));
    val[ci * kPadMaxK + t] = lnc[t] + 0.5f * (float)n * logf(s2 + c2 * P * P);
  }
  __syncthreads();
  for (int ci = tid; ci < kPadCandidates; ci += nt) {
    float mx = -INFINITY;
    for (int t = 0; t < T; ++t) mx = fmaxf(mx, val[ci * kPadMaxK + t]);
    float acc = 0.0f;
    for (int t = 0; t < T; ++t) acc += expf(val[ci * kPadMaxK + t] - mx);
    F[ci] = mx + logf(acc) - (float)k * (float)(e_lo + ci) * 0.6931471805599453f;
  }
  __syncthreads();
  int best = 0;
  for (int ci = 1; ci < kPadCandidates; ++ci)
    if (F[ci] < F[best]) best = ci;
  __syncthreads();
  const int e = e_lo + best;
  return e < -PAD_EXP_MAX ? -PAD_EXP_MAX : (e > PAD_EXP_MAX ? PAD_EXP_MAX : e);
}

}  // namespace permgpu
