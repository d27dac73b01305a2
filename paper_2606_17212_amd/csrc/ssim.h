// SSIM pieces shared by the utility and objective kernels: the 11x11
// Gaussian window (sigma 1.5), applied by the kernels as two 11-tap passes
// over an LDS tile with a 5-pixel apron, constants (0.01)^2 and (0.03)^2 for
// peak 1, zero padding outside the image.  Values are shifted by -0.5 before
// the moments are formed (inside the image and in the padding alike, so the
// shift is common to the whole window): variances and covariances do not
// change, and the shifted moments lose less to cancellation in FP32.
#pragma once

#include <math.h>

#include "common.h"

namespace dgs {

constexpr float kSsimC1 = 1.0e-4f;  // (0.01)^2
constexpr float kSsimC2 = 9.0e-4f;  // (0.03)^2
constexpr float kShift = 0.5f;
constexpr int kSsimR = 5;           // window radius

// Normalised 11-tap window (the 2D window is the outer product of two).
struct SsimWeights {
  float w[2 * kSsimR + 1];
};

// SSIM from shifted window moments.
__device__ __forceinline__ float ssim_value(float mx, float my, float exx, float eyy, float exy) {
  const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
  const float ux = mx + kShift, uy = my + kShift;
  const float num = (2.0f * ux * uy + kSsimC1) * (2.0f * sxy + kSsimC2);
  const float den = (ux * ux + uy * uy + kSsimC1) * (sxx + syy + kSsimC2);
  return num / den;
}

// Sum over the workgroup (every thread gets it).
__device__ __forceinline__ float block_sum(float v, float *red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Sum over the workgroup in a fixed order (FP64).
__device__ inline double block_sum_f64(double v, double *red) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// Normalised window taps (host).
inline SsimWeights ssim_weights() {
  SsimWeights W;
  double g[2 * kSsimR + 1], s = 0.0;
  for (int d = -kSsimR; d <= kSsimR; ++d) s += (g[d + kSsimR] = exp(-(double)(d * d) / (2.0 * 1.5 * 1.5)));
  for (int d = 0; d <= 2 * kSsimR; ++d) W.w[d] = (float)(g[d] / s);
  return W;
}

}  // namespace dgs
