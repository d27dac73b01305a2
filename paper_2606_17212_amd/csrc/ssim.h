// SSIM window statistics shared by the utility and objective kernels: the
// 11x11 Gaussian window (sigma 1.5) applied as two 11-tap passes over an LDS
// tile with a 5-pixel apron, constants (0.01)^2 and (0.03)^2 for peak 1, zero
// padding outside the image.  Values are shifted by -0.5 before the moments
// are formed (inside the image and in the padding alike, so the shift is
// common to the whole window): variances and covariances do not change, and
// the shifted moments lose less to cancellation in FP32.
#pragma once

#include <math.h>

#include "common.h"

namespace dgs {

constexpr float kSsimC1 = 1.0e-4f;  // (0.01)^2
constexpr float kSsimC2 = 9.0e-4f;  // (0.03)^2
constexpr float kShift = 0.5f;
constexpr int kSsimR = 5;           // window radius

// LDS of the window statistics of NX images against one reference, one
// channel at a time, for a TW x TH output block with a 5-pixel apron: the
// caller fills x and y (shifted values, apron row-major), ssim_moments then
// returns this thread's pixel's shifted window means and second moments.
template <int NX, int TW, int TH>
struct SsimLds {
  static constexpr int AW = TW + 2 * kSsimR, AH = TH + 2 * kSsimR, A = AW * AH;
  float x[NX][A];
  float y[A];
  // horizontal pass, rows [0, NX) mu_k, NX mu_y, [NX+1, 2NX+1) e_kk, 2NX+1 e_yy, [2NX+2, 3NX+2) e_ky
  float h[3 * NX + 2][AH * TW];
};

struct SsimWeights {
  float w[2 * kSsimR + 1];
};

template <int NX, int TW, int TH>
__device__ __forceinline__ void ssim_moments(SsimLds<NX, TW, TH> &L, const SsimWeights &W, float (&mu)[NX],
                                             float &muy, float (&ekk)[NX], float &eyy, float (&eky)[NX]) {
  using SL = SsimLds<NX, TW, TH>;
  // horizontal 11-tap pass over every apron row, for the TW output columns
  for (int q = threadIdx.x; q < SL::AH * TW; q += kBlock) {
    const int r = q / TW, cx = q % TW;
    float sm[NX], sk[NX], sky[NX], smy = 0.0f, syy = 0.0f;
#pragma unroll
    for (int k = 0; k < NX; ++k) sm[k] = sk[k] = sky[k] = 0.0f;
#pragma unroll
    for (int d = 0; d <= 2 * kSsimR; ++d) {
      const int a = r * SL::AW + cx + d;
      const float wd = W.w[d];
      const float yv = L.y[a];
      smy = fmaf(wd, yv, smy);
      syy = fmaf(wd, yv * yv, syy);
#pragma unroll
      for (int k = 0; k < NX; ++k) {
        const float xv = L.x[k][a];
        sm[k] = fmaf(wd, xv, sm[k]);
        sk[k] = fmaf(wd, xv * xv, sk[k]);
        sky[k] = fmaf(wd, xv * yv, sky[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      L.h[k][q] = sm[k];
      L.h[NX + 1 + k][q] = sk[k];
      L.h[2 * NX + 2 + k][q] = sky[k];
    }
    L.h[NX][q] = smy;
    L.h[2 * NX + 1][q] = syy;
  }
  __syncthreads();
  // vertical 11-tap pass for this thread's output pixel
  const int ox = threadIdx.x % TW, oy = threadIdx.x / TW;
  muy = eyy = 0.0f;
#pragma unroll
  for (int k = 0; k < NX; ++k) mu[k] = ekk[k] = eky[k] = 0.0f;
#pragma unroll
  for (int d = 0; d <= 2 * kSsimR; ++d) {
    const int q = (oy + d) * TW + ox;
    const float wd = W.w[d];
    muy = fmaf(wd, L.h[NX][q], muy);
    eyy = fmaf(wd, L.h[2 * NX + 1][q], eyy);
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      mu[k] = fmaf(wd, L.h[k][q], mu[k]);
      ekk[k] = fmaf(wd, L.h[NX + 1 + k][q], ekk[k]);
      eky[k] = fmaf(wd, L.h[2 * NX + 2 + k][q], eky[k]);
    }
  }
}

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
