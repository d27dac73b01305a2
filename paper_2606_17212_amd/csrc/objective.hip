// Packet-conditioned rendering objective (Sec. 4, Eq. (2)) and its image
// gradient, on the device:
//
//   L = E[D] + lambda_c CVaR_alpha(D) + lambda_t F + lambda_m M + lambda_a D_anchor
//
// D = MSE + lambda_ssim (1 - SSIM) per image against its target.  E and the
// upper-tail CVaR run over the partial states (the largest floor(alpha n)
// values count fully, the next one with the remainder, over alpha n; ties by
// list position); M averages max(0, D_b - D_a) over (a, b) pairs where b grows
// a's prefix; F averages, over (a, b) pairs of one world at two times, the
// mean squared error of the rendered change against the target change; the
// anchor term supervises complete-prefix states.  The rate proxy has weight 0
// in the configuration the paper locks and no dependence on the images.
//
// dL/dI_k = c_k dD_k/dI_k + the temporal terms, with c_k = dL/dD_k from the
// roles.  dSSIM/dx at pixel q is a sum over the windows that contain q: with
// per-pixel coefficients a = ds/du_x - 2 u'_x ds/ds_xx - u'_y ds/ds_xy,
// b = ds/ds_xx, c = ds/ds_xy (shifted means u', variance s_xx, covariance
// s_xy of the window around p),
//   dSSIM/dx(q) = (w * a)(q) + 2 x'(q) (w * b)(q) + y'(q) (w * c)(q),
// divided by 3 H W; * is the window correlation over image pixels (zero
// outside), x' and y' the shifted values.  The moments pass writes a, b, c;
// the gradient pass correlates them with the same two 11-tap passes.
//
// Kernels: k_obj_moments (per image and 16x16 block: window moments, SSIM,
// squared error, coefficient maps), k_obj_temporal (per pair and block:
// squared temporal-change error; the pair's two list entries), a radix sort of
// those entries by image, k_obj_dfinal (D per image), k_obj_weights (one
// workgroup: CVaR ranking, the loss parts, c_k, per-image pair offsets),
// k_obj_grad (per image and block: the gradient image).  Every sum has a fixed
// order, so results are reproducible bit for bit.
#include <math.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "objective.h"
#include "ssim.h"

namespace dgs {

ObjLayout make_obj_layout(int64_t K, int64_t width, int64_t height, int64_t Q) {
  ObjLayout L{};
  const int64_t blocks = ceil_div(width, 16) * ceil_div(height, 16);
  const int64_t kk = K > 0 ? K : 1, qq = Q > 0 ? Q : 1;
  const int64_t sort_blocks = sort_blocks_for(2 * qq);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  L.header = take(sizeof(ObjHeader));
  L.dpart = take(16 * kk * blocks);
  L.tpart = take(8 * qq * blocks);
  L.maps = take(4 * kk * 9 * width * height);
  L.cnt = take(4 * 5 * kk);
  L.coef = take(4 * kk);
  L.tcnt = take(4 * (kk + 1));
  L.tkey0 = take(8 * qq);
  L.tkey1 = take(8 * qq);
  L.tval0 = take(8 * qq);
  L.tval1 = take(8 * qq);
  L.thist = take(4 * 256 * sort_blocks);
  L.tparts = take(8 * (ceil_div(256 * sort_blocks, kScanTile) + 1));
  L.d = take(4 * kk);
  L.tsum = take(8 * qq);
  L.total = o;
  return L;
}

// ------------------------------------------------------------- moments
// One 16x16 block of one image.  The three channels of the 26x26 apron are
// read at once (12 contiguous bytes per pixel); then per channel the
// horizontal 11-tap pass of the five window sums (two adjacent output columns
// per task: 12 reads for 22 taps) and the vertical pass, SSIM and the
// coefficient maps.  One channel's horizontal sums at a time keep the
// workgroup at 24.5 KB of LDS (six per CU instead of three).
constexpr int kObjAW = 16 + 2 * kSsimR, kObjAH = 16 + 2 * kSsimR, kObjA = kObjAW * kObjAH;

// Horizontal 11-tap sums of rows r of `in` (apron layout) for output columns
// cx and cx + 1.
__device__ __forceinline__ void hpass2(const float *__restrict__ in, const SsimWeights &W, int r, int cx,
                                       float &o0, float &o1) {
  const float *row = in + r * kObjAW + cx;
  float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
  for (int d = 0; d <= 2 * kSsimR + 1; ++d) {
    const float v = row[d];
    if (d <= 2 * kSsimR) s0 = fmaf(W.w[d], v, s0);
    if (d >= 1) s1 = fmaf(W.w[d - 1], v, s1);
  }
  o0 = s0;
  o1 = s1;
}

__global__ void __launch_bounds__(kBlock) k_obj_moments(ObjArgs a, SsimWeights W) {
  __shared__ float xs[3][kObjA], ys[3][kObjA];
  // horizontal sums of one channel: x, y, xx, yy, xy over (26 rows x 16 columns)
  __shared__ float hs[5][kObjAH * 16];
  __shared__ float red[4];
  const int blk = blockIdx.x, k = blockIdx.y;
  const int tx = blk % a.bx, ty = blk / a.bx;
  const int64_t plane = (int64_t)a.width * a.height;
  const float *im = a.images + (int64_t)k * plane * 3;
  const int t = a.target_of[k];
  const bool tok = t >= 0 && t < a.T;
  if (!tok && threadIdx.x == 0) atomicOr(&a.hdr->bad, 1u);
  const float *tg = tok ? a.targets + (int64_t)t * plane * 3 : im;  // in bounds; the loss is NaN then
  const int x0 = tx * 16 - kSsimR, y0 = ty * 16 - kSsimR;
  for (int q = threadIdx.x; q < kObjA; q += kBlock) {
    const int gx = x0 + q % kObjAW, gy = y0 + q / kObjAW;
    float v0 = -kShift, v1 = -kShift, v2 = -kShift, w0 = -kShift, w1 = -kShift, w2 = -kShift;
    if (gx >= 0 && gx < a.width && gy >= 0 && gy < a.height) {
      const int64_t o = ((int64_t)gy * a.width + gx) * 3;
      v0 = im[o] - kShift; v1 = im[o + 1] - kShift; v2 = im[o + 2] - kShift;
      w0 = tg[o] - kShift; w1 = tg[o + 1] - kShift; w2 = tg[o + 2] - kShift;
    }
    xs[0][q] = v0; xs[1][q] = v1; xs[2][q] = v2;
    ys[0][q] = w0; ys[1][q] = w1; ys[2][q] = w2;
  }
  __syncthreads();
  const int ox = threadIdx.x % 16, oy = threadIdx.x / 16;
  const int px = tx * 16 + ox, py = ty * 16 + oy;
  const bool inpx = px < a.width && py < a.height;
  float se = 0.0f, ss = 0.0f;
  float mp[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    for (int task = threadIdx.x; task < kObjAH * 8; task += kBlock) {
      const int r = task / 8, cx = (task % 8) * 2;
      const float *xr = &xs[c][r * kObjAW + cx], *yr = &ys[c][r * kObjAW + cx];
      float m0 = 0, m1 = 0, n0 = 0, n1 = 0, p0 = 0, p1 = 0, q0 = 0, q1 = 0, s0 = 0, s1 = 0;
#pragma unroll
      for (int d = 0; d <= 2 * kSsimR + 1; ++d) {
        const float xv = xr[d], yv = yr[d];
        const float xx = xv * xv, yy = yv * yv, xy = xv * yv;
        if (d <= 2 * kSsimR) {
          const float wd = W.w[d];
          m0 = fmaf(wd, xv, m0); n0 = fmaf(wd, yv, n0); p0 = fmaf(wd, xx, p0); q0 = fmaf(wd, yy, q0);
          s0 = fmaf(wd, xy, s0);
        }
        if (d >= 1) {
          const float wd = W.w[d - 1];
          m1 = fmaf(wd, xv, m1); n1 = fmaf(wd, yv, n1); p1 = fmaf(wd, xx, p1); q1 = fmaf(wd, yy, q1);
          s1 = fmaf(wd, xy, s1);
        }
      }
      const int o = r * 16 + cx;
      hs[0][o] = m0; hs[0][o + 1] = m1;
      hs[1][o] = n0; hs[1][o + 1] = n1;
      hs[2][o] = p0; hs[2][o + 1] = p1;
      hs[3][o] = q0; hs[3][o + 1] = q1;
      hs[4][o] = s0; hs[4][o + 1] = s1;
    }
    __syncthreads();
    if (inpx) {
      float mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
#pragma unroll
      for (int d = 0; d <= 2 * kSsimR; ++d) {
        const int q = (oy + d) * 16 + ox;
        const float wd = W.w[d];
        mx = fmaf(wd, hs[0][q], mx);
        my = fmaf(wd, hs[1][q], my);
        exx = fmaf(wd, hs[2][q], exx);
        eyy = fmaf(wd, hs[3][q], eyy);
        exy = fmaf(wd, hs[4][q], exy);
      }
      const int ai = (oy + kSsimR) * kObjAW + ox + kSsimR;
      const float dv = xs[c][ai] - ys[c][ai];
      se += dv * dv;
      const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
      const float ux = mx + kShift, uy = my + kShift;
      const float A1 = 2.0f * ux * uy + kSsimC1, A2 = 2.0f * sxy + kSsimC2;
      const float B1 = ux * ux + uy * uy + kSsimC1, B2 = sxx + syy + kSsimC2;
      const float sv = (A1 * A2) / (B1 * B2);
      ss += sv;
      const float inv = 1.0f / (B1 * B2);
      const float ds_ux = 2.0f * uy * A2 * inv - sv * (2.0f * ux) / B1;
      const float ds_sxx = -sv / B2;
      const float ds_sxy = 2.0f * A1 * inv;
      mp[3 * c] = ds_ux - 2.0f * mx * ds_sxx - my * ds_sxy;
      mp[3 * c + 1] = ds_sxx;
      mp[3 * c + 2] = ds_sxy;
    }
    __syncthreads();  // the next channel overwrites the horizontal sums
  }
  if (inpx) {
    float *dst = a.maps + ((int64_t)k * plane + (int64_t)py * a.width + px) * 9;
#pragma unroll
    for (int j = 0; j < 9; ++j) dst[j] = mp[j];
  }
  const float tse = block_sum(se, red);
  const float tss = block_sum(ss, red);
  if (threadIdx.x == 0) {
    const int64_t o = ((int64_t)k * a.bx * a.by + blk) * 2;
    a.dpart[o] = (double)tse;
    a.dpart[o + 1] = (double)tss;
  }
}

// ------------------------------------------------------------ temporal
// Pair j = (a, b): sum over the block of ((I_b - I_a) - (G_b - G_a))^2; the
// first block also writes the pair's two entries for the per-image sort (an
// invalid pair sorts after every image).
__global__ void __launch_bounds__(kBlock) k_obj_temporal(ObjArgs a) {
  __shared__ float red[4];
  const int blk = blockIdx.x, j = blockIdx.y;
  const int tx = blk % a.bx, ty = blk / a.bx;
  const int ia = a.temporal[2 * j], ib = a.temporal[2 * j + 1];
  bool ok = ia >= 0 && ia < a.K && ib >= 0 && ib < a.K;
  const int ta = ok ? a.target_of[ia] : 0, tb = ok ? a.target_of[ib] : 0;
  ok = ok && ta >= 0 && ta < a.T && tb >= 0 && tb < a.T;
  if (blk == 0 && threadIdx.x == 0) {
    if (!ok) atomicOr(&a.hdr->bad, 1u);
    a.tkey0[2 * j] = ok ? (uint32_t)ia : (uint32_t)a.K;
    a.tkey0[2 * j + 1] = ok ? (uint32_t)ib : (uint32_t)a.K;
    a.tval0[2 * j] = ((uint32_t)j << 1) | 0u;
    a.tval0[2 * j + 1] = ((uint32_t)j << 1) | 1u;
  }
  if (!ok) {  // uniform over the workgroup
    if (threadIdx.x == 0) a.tpart[(int64_t)j * a.bx * a.by + blk] = 0.0;
    return;
  }
  const int64_t plane = (int64_t)a.width * a.height;
  const int px = tx * 16 + threadIdx.x % 16, py = ty * 16 + threadIdx.x / 16;
  float s = 0.0f;
  if (px < a.width && py < a.height) {
    const int64_t o = (int64_t)py * a.width + px;
    const float *xa = a.images + ((int64_t)ia * plane + o) * 3, *xb = a.images + ((int64_t)ib * plane + o) * 3;
    const float *ga = a.targets + ((int64_t)ta * plane + o) * 3, *gb = a.targets + ((int64_t)tb * plane + o) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float e = (xb[c] - xa[c]) - (gb[c] - ga[c]);
      s += e * e;
    }
  }
  const float tot = block_sum(s, red);
  if (threadIdx.x == 0) a.tpart[(int64_t)j * a.bx * a.by + blk] = (double)tot;
}

// D per image (workgroups 0..K-1) and the squared temporal-change error per
// pair (workgroups K..K+Q-1), each summed over the 16x16 blocks in a fixed order.
__global__ void __launch_bounds__(kBlock) k_obj_dfinal(ObjArgs a) {
  __shared__ double red[4];
  const int blocks = a.bx * a.by;
  if ((int)blockIdx.x >= a.K) {
    const int j = blockIdx.x - a.K;
    double s = 0.0;
    for (int b = threadIdx.x; b < blocks; b += kBlock) s += a.tpart[(int64_t)j * blocks + b];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) a.tsum[j] = s;
    return;
  }
  const int k = blockIdx.x;
  double se = 0.0, ss = 0.0;
  for (int b = threadIdx.x; b < blocks; b += kBlock) {
    se += a.dpart[((int64_t)k * blocks + b) * 2];
    ss += a.dpart[((int64_t)k * blocks + b) * 2 + 1];
  }
  se = block_sum_f64(se, red);
  ss = block_sum_f64(ss, red);
  if (threadIdx.x == 0) {
    const double n3 = 3.0 * (double)a.width * (double)a.height;
    const float d = (float)(se / n3 + (double)a.w.lambda_ssim * (1.0 - ss / n3));
    a.d[k] = d;
    if (a.distortion) a.distortion[k] = d;
  }
}

// ------------------------------------------------------------- weights
// Counters updated by atomics in this workgroup are read back at device
// scope (the atomics act in L2; a plain load could see a stale L1 line).
__device__ __forceinline__ int load_l2(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Monotone unsigned key of a float (larger value -> larger key).
__device__ __forceinline__ uint32_t ordered_bits(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void __launch_bounds__(kBlock) k_obj_weights(ObjArgs a) {
  __shared__ unsigned long long key[kObjMaxExpect];
  __shared__ double red[4];
  __shared__ int s_bad;
  const int tid = threadIdx.x, K = a.K;
  int *cE = a.cnt, *cT = a.cnt + K, *cB = a.cnt + 2 * K, *cA = a.cnt + 3 * K, *cM = a.cnt + 4 * K;
  for (int i = tid; i < 5 * K; i += kBlock) a.cnt[i] = 0;
  for (int i = tid; i <= K; i += kBlock) a.tcnt[i] = 0;
  if (tid == 0) s_bad = (int)a.hdr->bad;
  __syncthreads();
  int bad = 0;
  // partial states: E and the ranking for the tail (descending D, then list position)
  const int nE = a.n_expect;
  int P2 = 1;
  while (P2 < nE) P2 <<= 1;
  double sE = 0.0;
  for (int i = tid; i < P2; i += kBlock) {
    unsigned long long kk = ~0ull;
    if (i < nE) {
      const int idx = a.expect[i];
      if (idx >= 0 && idx < K) {
        const float v = a.d[idx];
        sE += (double)v;
        atomicAdd(&cE[idx], 1);
        kk = ((unsigned long long)(~ordered_bits(v)) << 32) | (unsigned long long)i;
      } else {
        bad = 1;
      }
    }
    key[i] = kk;
  }
  __syncthreads();
  for (int k2 = 2; k2 <= P2; k2 <<= 1)
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P2; i += kBlock) {
        const int l = i ^ j;
        if (l > i) {
          const unsigned long long x = key[i], y = key[l];
          if ((x > y) == ((i & k2) == 0)) { key[i] = y; key[l] = x; }
        }
      }
      __syncthreads();
    }
  const double an = (double)a.w.alpha * (double)nE;
  const int kt = (int)floor(an);
  const double frac = an - (double)kt;
  double sT = 0.0;
  for (int r = tid; r < nE; r += kBlock) {
    const unsigned long long kk = key[r];
    if (kk == ~0ull) continue;  // an invalid entry (flagged above)
    const int idx = a.expect[(int)(kk & 0xFFFFFFFFull)];
    if (r < kt) {
      sT += (double)a.d[idx];
      atomicAdd(&cT[idx], 1);
    } else if (r == kt && frac > 0.0) {
      sT += frac * (double)a.d[idx];
      atomicAdd(&cB[idx], 1);
    }
  }
  double sA = 0.0;
  for (int i = tid; i < a.n_anchor; i += kBlock) {
    const int idx = a.anchor[i];
    if (idx >= 0 && idx < K) {
      sA += (double)a.d[idx];
      atomicAdd(&cA[idx], 1);
    } else {
      bad = 1;
    }
  }
  double sM = 0.0;
  for (int i = tid; i < a.n_mono; i += kBlock) {
    const int ia = a.mono[2 * i], ib = a.mono[2 * i + 1];
    if (ia < 0 || ia >= K || ib < 0 || ib >= K) { bad = 1; continue; }
    const float da = a.d[ia], db = a.d[ib];
    if (db > da) {  // a quality regression as the prefix grows (no gradient at equality)
      sM += (double)db - (double)da;
      atomicAdd(&cM[ib], 1);
      atomicAdd(&cM[ia], -1);
    }
  }
  double sF = 0.0;
  for (int j = tid; j < a.n_temporal; j += kBlock) {
    const int ia = a.temporal[2 * j], ib = a.temporal[2 * j + 1];
    if (ia < 0 || ia >= K || ib < 0 || ib >= K) continue;  // flagged by k_obj_temporal
    const int ta = a.target_of[ia], tb = a.target_of[ib];
    if (ta < 0 || ta >= a.T || tb < 0 || tb >= a.T) continue;  // likewise
    sF += a.tsum[j];
    atomicAdd(&a.tcnt[ia], 1);
    atomicAdd(&a.tcnt[ib], 1);
  }
  if (bad) atomicOr(&s_bad, 1);
  sE = block_sum_f64(sE, red);
  sT = block_sum_f64(sT, red);
  sA = block_sum_f64(sA, red);
  sM = block_sum_f64(sM, red);
  sF = block_sum_f64(sF, red);  // also orders the count atomics above before their reads below
  const bool any_bad = s_bad != 0;
  const double n3 = 3.0 * (double)a.width * (double)a.height;
  const double E = nE ? sE / nE : 0.0, CV = nE ? sT / an : 0.0, A = a.n_anchor ? sA / a.n_anchor : 0.0;
  const double M = a.n_mono ? sM / a.n_mono : 0.0, F = a.n_temporal ? sF / ((double)a.n_temporal * n3) : 0.0;
  const ObjWeights &w = a.w;
  if (tid == 0) {
    const double Lv = E + w.lambda_c * CV + w.lambda_t * F + w.lambda_m * M + w.lambda_a * A;
    const float nan = __int_as_float(0x7FC00000);
    a.loss[0] = any_bad ? nan : (float)Lv;
    a.loss[1] = any_bad ? nan : (float)E;
    a.loss[2] = any_bad ? nan : (float)CV;
    a.loss[3] = any_bad ? nan : (float)F;
    a.loss[4] = any_bad ? nan : (float)M;
    a.loss[5] = any_bad ? nan : (float)A;
    if (any_bad) atomicOr(&a.hdr->bad, 1u);
  }
  for (int k = tid; k < K; k += kBlock) {
    double c = 0.0;
    if (nE) c += load_l2(&cE[k]) / (double)nE + w.lambda_c * (load_l2(&cT[k]) + frac * load_l2(&cB[k])) / an;
    if (a.n_anchor) c += w.lambda_a * load_l2(&cA[k]) / (double)a.n_anchor;
    if (a.n_mono) c += w.lambda_m * load_l2(&cM[k]) / (double)a.n_mono;
    a.coef[k] = any_bad ? __int_as_float(0x7FC00000) : (float)c;
  }
  // per-image offsets of the temporal entries: exclusive scan of tcnt[0..K)
  // (each thread scans a contiguous chunk; chunk totals scanned by thread 0)
  __syncthreads();
  __shared__ int chunk[kBlock];
  const int per = (K + kBlock - 1) / kBlock;
  const int c0 = tid * per, c1 = min(K, c0 + per);
  int run = 0;
  for (int i = c0; i < c1; ++i) run += load_l2(&a.tcnt[i]);
  chunk[tid] = run;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int i = 0; i < kBlock; ++i) { const int v = chunk[i]; chunk[i] = acc; acc += v; }
  }
  __syncthreads();
  int acc = chunk[tid];
  for (int i = c0; i < c1; ++i) { const int v = load_l2(&a.tcnt[i]); a.tcnt[i] = acc; acc += v; }
  if (tid == kBlock - 1) a.tcnt[K] = acc;
}

// --------------------------------------------------------------- gradient
// One 16x16 block of one image: the nine coefficient maps of the apron at
// once (36 contiguous bytes per pixel), the horizontal pass of all nine with
// two output columns per task, then per channel the vertical pass and the
// gradient.  Two barriers.
__global__ void __launch_bounds__(kBlock) k_obj_grad(ObjArgs a, SsimWeights W, const uint32_t *__restrict__ tvals) {
  __shared__ float m[9][kObjA];
  __shared__ float hp[9][kObjAH * 16];
  const int blk = blockIdx.x, k = blockIdx.y;
  const int tx = blk % a.bx, ty = blk / a.bx;
  const int64_t plane = (int64_t)a.width * a.height;
  const int ox = threadIdx.x % 16, oy = threadIdx.x / 16;
  const int px = tx * 16 + ox, py = ty * 16 + oy;
  const bool in = px < a.width && py < a.height;
  const int64_t o = (int64_t)py * a.width + px;
  const float ck = a.coef[k];
  const int e0 = a.tcnt[k], e1 = a.tcnt[k + 1];
  const bool ssim_part = ck != 0.0f;  // NaN (invalid lists) takes this path too
  const int t = a.target_of[k];
  const bool tok = t >= 0 && t < a.T;
  const double n3 = 3.0 * (double)plane;
  const float inv3n = (float)(1.0 / n3);
  const float ct = a.n_temporal ? (float)(2.0 * (double)a.w.lambda_t / ((double)a.n_temporal * n3)) : 0.0f;
  const int x0 = tx * 16 - kSsimR, y0 = ty * 16 - kSsimR;
  float g[3] = {0.0f, 0.0f, 0.0f};
  if (ssim_part) {  // uniform over the workgroup
    for (int q = threadIdx.x; q < kObjA; q += kBlock) {
      const int gx = x0 + q % kObjAW, gy = y0 + q / kObjAW;
      float v[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) v[j] = 0.0f;
      if (gx >= 0 && gx < a.width && gy >= 0 && gy < a.height) {
        const float *src = a.maps + ((int64_t)k * plane + (int64_t)gy * a.width + gx) * 9;
#pragma unroll
        for (int j = 0; j < 9; ++j) v[j] = src[j];
      }
#pragma unroll
      for (int j = 0; j < 9; ++j) m[j][q] = v[j];
    }
    __syncthreads();
    for (int task = threadIdx.x; task < 9 * kObjAH * 8; task += kBlock) {
      const int j = task / (kObjAH * 8), rem = task % (kObjAH * 8), r = rem / 8, cx = (rem % 8) * 2;
      float h0, h1;
      hpass2(m[j], W, r, cx, h0, h1);
      hp[j][r * 16 + cx] = h0;
      hp[j][r * 16 + cx + 1] = h1;
    }
    __syncthreads();
    if (in && tok) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float wa = 0.0f, wb = 0.0f, wc = 0.0f;
#pragma unroll
        for (int d = 0; d <= 2 * kSsimR; ++d) {
          const int q = (oy + d) * 16 + ox;
          wa = fmaf(W.w[d], hp[3 * c][q], wa);
          wb = fmaf(W.w[d], hp[3 * c + 1][q], wb);
          wc = fmaf(W.w[d], hp[3 * c + 2][q], wc);
        }
        const float x = a.images[((int64_t)k * plane + o) * 3 + c];
        const float y = a.targets[((int64_t)t * plane + o) * 3 + c];
        const float xs = x - kShift, ys = y - kShift;
        const float dssim = (wa + 2.0f * xs * wb + ys * wc) * inv3n;
        g[c] = ck * (2.0f * (x - y) * inv3n - a.w.lambda_ssim * dssim);
      }
    } else if (in) {
      g[0] = g[1] = g[2] = ck;  // invalid target: NaN like the loss
    }
  }
  if (!in) return;
  for (int e = e0; e < e1; ++e) {
    const uint32_t v = tvals[e];
    const int j = (int)(v >> 1);
    const int ia = a.temporal[2 * j], ib = a.temporal[2 * j + 1];
    const int ta = a.target_of[ia], tb = a.target_of[ib];
    const float *xa = a.images + ((int64_t)ia * plane + o) * 3, *xb = a.images + ((int64_t)ib * plane + o) * 3;
    const float *ga = a.targets + ((int64_t)ta * plane + o) * 3, *gb = a.targets + ((int64_t)tb * plane + o) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float ev = (xb[c] - xa[c]) - (gb[c] - ga[c]);
      g[c] += (v & 1u) ? ct * ev : -ct * ev;
    }
  }
  float *dst = a.grad + ((int64_t)k * plane + o) * 3;
  dst[0] = g[0];
  dst[1] = g[1];
  dst[2] = g[2];
}

__global__ void k_obj_clear(ObjHeader *h) {
  if (threadIdx.x == 0) h->bad = 0u;
}

// ------------------------------------------------------------------ L1 loss
// L = sum_k sum_j |x_kj - t_{target_of[k], j}| / (K n), n = H W 3 elements per
// image.  Partials in FP64, summed in a fixed order: the loss does not depend
// on scheduling.  An out-of-range target index sets the header's flag and
// makes the loss (and that image's gradient) NaN; nothing is read out of
// bounds.

size_t l1_scratch_bytes(int64_t K, int64_t width, int64_t height) {
  const int64_t chunks = ceil_div(width * height * 3, kL1Chunk);
  return align256(sizeof(ObjHeader)) + align256(8 * (K > 0 ? K : 1) * chunks);
}

__device__ inline bool l1_target(const int32_t *target_of, int k, int T, int &t) {
  t = target_of ? target_of[k] : 0;
  return t >= 0 && t < T;
}

__global__ void __launch_bounds__(kBlock)
k_l1_partial(const float *__restrict__ x, int64_t n, const float *__restrict__ tg, int T,
             const int32_t *__restrict__ target_of, ObjHeader *h, double *__restrict__ part) {
  const int k = blockIdx.y;
  int t;
  const bool ok = l1_target(target_of, k, T, t);
  const int64_t j0 = (int64_t)blockIdx.x * kL1Chunk;
  float s = 0.0f;
  if (ok) {
    const float *xi = x + (int64_t)k * n, *ti = tg + (int64_t)t * n;
#pragma unroll 4
    for (int64_t j = j0 + threadIdx.x; j < j0 + kL1Chunk && j < n; j += kBlock) s += fabsf(xi[j] - ti[j]);
  }
  double d = s;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, kWave);
  __shared__ double w[4];
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    part[(int64_t)k * gridDim.x + blockIdx.x] = ok ? ((w[0] + w[1]) + (w[2] + w[3])) : __longlong_as_double(0x7FF8000000000000LL);
    if (!ok) atomicOr(&h->bad, 1u);
  }
}

__global__ void __launch_bounds__(1024) k_l1_finalize(const double *__restrict__ part, int64_t np, double inv,
                                                      float *loss) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += 1024) s += part[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
  __shared__ double w[16];
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 16; ++i) t += w[i];
    loss[0] = (float)(t * inv);
  }
}

__global__ void k_l1_clear(ObjHeader *h, float *loss, int empty) {
  if (threadIdx.x == 0) {
    h->bad = 0u;
    if (empty) loss[0] = 0.0f;
  }
}

void launch_l1_loss(const float *images, int K, int64_t per_image, const float *targets, int T,
                    const int32_t *target_of, float *loss, void *scratch, hipStream_t st) {
  ObjHeader *h = reinterpret_cast<ObjHeader *>(scratch);
  double *part = reinterpret_cast<double *>(reinterpret_cast<char *>(scratch) + align256(sizeof(ObjHeader)));
  const int64_t chunks = ceil_div(per_image, kL1Chunk);
  k_l1_clear<<<1, 64, 0, st>>>(h, loss, K == 0 ? 1 : 0);
  if (K == 0) return;
  k_l1_partial<<<dim3((unsigned)chunks, (unsigned)K), kBlock, 0, st>>>(images, per_image, targets, T, target_of, h,
                                                                         part);
  k_l1_finalize<<<1, 1024, 0, st>>>(part, chunks * K, 1.0 / ((double)K * (double)per_image), loss);
}

// dL/dx = dloss sign(x - t) / (K n), sign(0) = 0; dloss NULL means 1.
__global__ void __launch_bounds__(kBlock)
k_l1_grad(const float *__restrict__ x, int64_t n, const float *__restrict__ tg, int T,
          const int32_t *__restrict__ target_of, const float *dloss, float inv, float *__restrict__ g) {
  const int k = blockIdx.y;
  int t;
  const bool ok = l1_target(target_of, k, T, t);
  const float sc = (dloss ? dloss[0] : 1.0f) * inv;
  const int64_t j0 = (int64_t)blockIdx.x * kL1Chunk;
  const float *xi = x + (int64_t)k * n, *ti = tg + (int64_t)(ok ? t : 0) * n;
  float *gi = g + (int64_t)k * n;
#pragma unroll 4
  for (int64_t j = j0 + threadIdx.x; j < j0 + kL1Chunk && j < n; j += kBlock) {
    if (!ok) {
      gi[j] = __int_as_float(0x7FC00000);
      continue;
    }
    const float d = xi[j] - ti[j];
    gi[j] = d > 0.0f ? sc : (d < 0.0f ? -sc : 0.0f);
  }
}

void launch_l1_grad(const float *images, int K, int64_t per_image, const float *targets, int T,
                    const int32_t *target_of, const float *dloss, float *grad, hipStream_t st) {
  if (K == 0) return;
  const int64_t chunks = ceil_div(per_image, kL1Chunk);
  k_l1_grad<<<dim3((unsigned)chunks, (unsigned)K), kBlock, 0, st>>>(
      images, per_image, targets, T, target_of, dloss, (float)(1.0 / ((double)K * (double)per_image)), grad);
}

// ---------------------------------------------------------------- launcher
void launch_objective(const ObjArgs &a, hipStream_t st) {
  const SsimWeights W = ssim_weights();
  const int blocks = a.bx * a.by;
  k_obj_clear<<<1, 64, 0, st>>>(a.hdr);
  if (a.K > 0) k_obj_moments<<<dim3(blocks, a.K), kBlock, 0, st>>>(a, W);
  const uint32_t *tvals = a.tval0;
  if (a.n_temporal > 0) {
    k_obj_temporal<<<dim3(blocks, a.n_temporal), kBlock, 0, st>>>(a);
    int bits = 1;
    while ((1 << bits) <= a.K) ++bits;  // keys 0..K (K = invalid pair)
    const int r = launch_radix_sort(a.tkey0, a.tval0, a.tkey1, a.tval1, nullptr, 0, 2 * (int64_t)a.n_temporal,
                                    0, bits, a.thist, a.tparts, st, /*last_pass_keys=*/false);
    tvals = r ? a.tval1 : a.tval0;
  }
  if (a.K + a.n_temporal > 0) k_obj_dfinal<<<a.K + a.n_temporal, kBlock, 0, st>>>(a);
  k_obj_weights<<<1, kBlock, 0, st>>>(a);
  if (a.K > 0 && a.grad) k_obj_grad<<<dim3(blocks, a.K), kBlock, 0, st>>>(a, W, tvals);
}

}  // namespace dgs
