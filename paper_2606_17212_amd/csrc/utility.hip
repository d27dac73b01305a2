// Counterfactual render utility (paper Sec. 5): Eq. (3)
//   Delta_g(m) = D(I, R(m)) - D(I, R(m u g)),  D = MSE + lambda (1 - SSIM)
// (the distortion fixed for the objective in Sec. 4), and the risk-adjusted
// utility of Eq. (4) over the contexts of each group.
//
// R(m) and R(m u g) differ only in pixels that a Gaussian of the completion
// group g = (packet, layer) reaches, i.e. inside the tiles of g's Gaussians'
// rectangles (the "core").  SSIM at a pixel depends on the 11x11 window around
// it, so the SSIM term can change only within 5 px of the core, and those
// pixels' windows lie within 10 px of the core.  The paired renderer
// therefore composites, for each context, only the "region" = core dilated by
// enough tiles to cover 10 px, both states at once (up to four contexts of one
// group share a workgroup as one 8-state group), and sums the per-pixel
// differences there.  Pixels of the region whose window
// reaches outside it see the same (zero) values in both states and so add
// exactly zero.  Delta is that sum over all pixels and channels divided by
// 3 H W.
//
// The SSIM windows are the 11x11 Gaussian (sigma 1.5) applied as two 11-tap
// passes; image values are shifted by -0.5 before the moments are formed
// (variances and covariances do not change under a common shift, and the
// shifted moments lose less to cancellation in FP32).

#include <math.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"
#include "ssim.h"

namespace dgs {

// ------------------------------------------------------------------ groups
__global__ void k_group_table(const uint16_t *__restrict__ group_pl, int G, int P, int *__restrict__ pl2g,
                              UtilHeader *h) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= G) return;
  const uint32_t pl = group_pl[k];
  if ((int)(pl >> 2) >= P) {
    atomicOr(&h->bad_group, 1u);
    return;
  }
  if (atomicCAS(&pl2g[pl], -1, k) != -1) atomicOr(&h->bad_group, 2u);  // two groups name one (packet, layer)
}

// Core tiles of every group: the tile rectangles of its Gaussians (with
// refinement levels: of its packet's records at depths layer - 1 and layer,
// the records that adding the group hides and shows).  Each row
// of a rectangle is a run of consecutive tile bits, set with one OR per
// bitmap word it touches.  LDS: the group bitmaps of all groups, privatised
// per workgroup and merged into the global ones once (when they fit).
constexpr int kCoreLdsWords = 8192;

__device__ __forceinline__ void mark_rect_rows(uint32_t *row, int tiles_x, int x0, int y0, int x1, int y1) {
  for (int y = y0; y < y1; ++y) {
    const int t0 = y * tiles_x + x0, t1 = y * tiles_x + x1 - 1;  // inclusive bit range
    for (int w = t0 >> 5; w <= (t1 >> 5); ++w) {
      const int lo = w == (t0 >> 5) ? (t0 & 31) : 0, hi = w == (t1 >> 5) ? (t1 & 31) : 31;
      const uint32_t m = (hi == 31 ? 0xFFFFFFFFu : ((1u << (hi + 1)) - 1u)) & ~((1u << lo) - 1u);
      atomicOr(row + w, m);
    }
  }
}

template <bool LDS>
__global__ void __launch_bounds__(kBlock)
k_group_core(const float4 *__restrict__ rec0, const uint2 *__restrict__ rect, int n, const int *__restrict__ pl2g,
             int tiles_x, int words, int gw, int refined, uint32_t *__restrict__ core) {
  __shared__ uint32_t bm[LDS ? kCoreLdsWords : 1];
  if (LDS) {
    for (int i = threadIdx.x; i < gw; i += kBlock) bm[i] = 0u;
    __syncthreads();
  }
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const uint2 r = rect[i];
    const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16;
    if (x1 <= x0 || y1 <= y0) continue;
    const uint32_t pl = __float_as_uint(rec0[i].w) & 0xFFFFu;
    const int g = pl2g[pl];
    // a record of depth d also changes when group (packet, d + 1) is added
    const int g2 = (refined && (pl & 3u) < 3u) ? pl2g[pl + 1] : -1;
    if (g >= 0) mark_rect_rows((LDS ? bm : core) + (int64_t)g * words, tiles_x, x0, y0, x1, y1);
    if (g2 >= 0) mark_rect_rows((LDS ? bm : core) + (int64_t)g2 * words, tiles_x, x0, y0, x1, y1);
  }
  if (LDS) {
    __syncthreads();
    for (int i = threadIdx.x; i < gw; i += kBlock) {
      const uint32_t v = bm[i];
      if (v) atomicOr(core + i, v);
    }
  }
}

__device__ __forceinline__ bool bit_at(const uint32_t *row, int t) { return (row[t >> 5] >> (t & 31)) & 1u; }

// Region = core dilated by (rx, ry) tiles; one thread per (group, 32-tile word).
__global__ void __launch_bounds__(kBlock)
k_group_region(const uint32_t *__restrict__ core, int G, int tiles_x, int tiles_y, int words, int rx, int ry,
               uint32_t *__restrict__ region, uint32_t *__restrict__ wcount) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= (int64_t)G * words) return;
  const int g = (int)(id / words), w = (int)(id % words);
  const uint32_t *row = core + (int64_t)g * words;
  const int tiles = tiles_x * tiles_y;
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    const int t = w * 32 + b;
    if (t >= tiles) break;
    const int tx = t % tiles_x, ty = t / tiles_x;
    bool any = false;
    for (int dy = -ry; dy <= ry && !any; ++dy) {
      const int yy = ty + dy;
      if (yy < 0 || yy >= tiles_y) continue;
      for (int dx = -rx; dx <= rx; ++dx) {
        const int xx = tx + dx;
        if (xx >= 0 && xx < tiles_x && bit_at(row, yy * tiles_x + xx)) {
          any = true;
          break;
        }
      }
    }
    bits |= (any ? 1u : 0u) << b;
  }
  region[id] = bits;
  wcount[id] = (uint32_t)__popc(bits);
}

// Tiles of every region in tile order: slot = exclusive word prefix + bits below.
__global__ void __launch_bounds__(kBlock)
k_region_tiles(const uint32_t *__restrict__ region, const uint32_t *__restrict__ wprefix, int64_t gw,
               int words, uint32_t *__restrict__ rtiles) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= gw) return;
  uint32_t bits = region[id];
  uint32_t o = wprefix[id];
  const int w = (int)(id % words);
  while (bits) {
    const int b = __ffs(bits) - 1;
    bits &= bits - 1;
    rtiles[o++] = (uint32_t)(w * 32 + b);
  }
}

// First region tile of each group (group_base[G] = total) from the word prefix.
__global__ void k_group_base(const uint32_t *__restrict__ wprefix, const unsigned long long *total, int G, int words,
                             uint32_t *__restrict__ gbase) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) gbase[g] = wprefix[(int64_t)g * words];
  if (g == G) gbase[G] = (uint32_t)*total;
}

// Work items per context (its group's region size) and the pair delivery
// bits: bit 0 for m, bit 1 for m u g.  A context must hold the group's packet
// at prefix depth exactly the group's layer.
__global__ void __launch_bounds__(kBlock)
k_pair_setup(const uint8_t *__restrict__ codes, const int32_t *__restrict__ context_group,
             const uint16_t *__restrict__ group_pl, const uint32_t *__restrict__ gbase, int J, int G, int P,
             uint32_t *__restrict__ icount, uint32_t *__restrict__ pvis, uint32_t *__restrict__ bad,
             UtilHeader *h, int exact) {
  const int j = blockIdx.x;
  if (j >= J) return;
  const int g = context_group[j];
  const bool gok = g >= 0 && g < G;
  const uint32_t gpl = gok ? group_pl[g] : 0u;
  const int gp = (int)(gpl >> 2), gl = (int)(gpl & 3u);
  const uint8_t *row = codes + (int64_t)j * P;
  const bool ok = gok && gp < P && row[gp] == gl;
  if (threadIdx.x == 0) {
    icount[j] = ok ? gbase[g + 1] - gbase[g] : 0u;
    bad[j] = ok ? 0u : 1u;
    if (!ok) atomicOr(&h->bad_context, 1u);
  }
  uint32_t *out = pvis + (int64_t)j * P * 4;
  for (int e = threadIdx.x; e < P * 4; e += kBlock) {
    const int p = e >> 2, l = e & 3;
    const int c = row[p];
    const int cg = (ok && p == gp) ? gl + 1 : c;
    if (exact)  // records at delivered depth l: shown where the state delivers exactly depth l
      out[e] = ((c < 4 ? c : 4) == l + 1 ? 1u : 0u) | ((cg < 4 ? cg : 4) == l + 1 ? 2u : 0u);
    else
      out[e] = (l < c ? 1u : 0u) | (l < cg ? 2u : 0u);
  }
}

// Compositing items of each bundle: its group's region tiles, counted at the
// context that starts it.
__global__ void __launch_bounds__(kBlock)
k_bundle_setup(const int32_t *__restrict__ context_group, const uint32_t *__restrict__ bad,
               const uint32_t *__restrict__ icount, int J, uint32_t *__restrict__ bcount) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= J) return;
  bcount[j] = (bad[j] == 0u && bundle_start(context_group, bad, j)) ? icount[j] : 0u;
}

// Pair items: per-pixel  sum_c (x1 - y)^2 - (x2 - y)^2 - lambda (ssim1 - ssim2)
// over the item's tile, for items whose 3x3 tile neighbourhood meets the core.
// One pass reads the apron of both states (from the neighbouring items'
// patches) and of the reference for all three channels; the horizontal
// 11-tap pass of the eight window sums runs per channel with two output
// columns per task.
template <int TW, int TH>
__global__ void __launch_bounds__(kBlock)
k_pair_ssim(UtilArgs u, SsimWeights W) {
  constexpr int AW = TW + 2 * kSsimR, AH = TH + 2 * kSsimR, A = AW * AH;
  __shared__ float xs[2][3][A];  // both states, shifted
  __shared__ float ys[3][A];     // reference, shifted
  // horizontal sums of one channel: x1, x2, y, x1^2, x2^2, y^2, x1 y, x2 y
  __shared__ float hs[8][AH * TW];
  __shared__ float red[4];
  __shared__ int s_item;
  const unsigned long long total = *u.item_total;
  const uint32_t n_items = total <= u.item_capacity ? (uint32_t)total : 0u;  // nothing after an overflow
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(u.queue, 1u);
    __syncthreads();
    const uint32_t item = (uint32_t)s_item;
    __syncthreads();
    if (item >= n_items) break;
    int lo = 0, hi = u.num_contexts - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (u.item_base[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const int j = lo;
    const int g = u.context_group[j];
    const int tile = (int)u.region_tiles[u.group_base[g] + (item - u.item_base[j])];
    const int tx = tile % u.tiles_x, ty = tile / u.tiles_x;
    const uint32_t *crow = u.core + (int64_t)g * u.words;
    const uint32_t *rrow = u.region + (int64_t)g * u.words;
    const uint32_t *rpre = u.wprefix + (int64_t)g * u.words;
    int near = 0;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int xx = tx + dx, yy = ty + dy;
        if (xx >= 0 && xx < u.tiles_x && yy >= 0 && yy < u.tiles_y && bit_at(crow, yy * u.tiles_x + xx)) near = 1;
      }
    // Without a core tile in the 3x3 neighbourhood every window of this tile
    // sees identical values in both states: the item adds zero.  The branch
    // is made wave-uniform explicitly and every path reaches the same
    // barriers (no early continue: a thread-0-only store before a jump back
    // to the barrier that publishes the next item can let the other lanes
    // re-read the old item).
    near = __builtin_amdgcn_readfirstlane(near);
    const int x0 = tx * TW - kSsimR, y0 = ty * TH - kSsimR;
    float acc = 0.0f;
    if (near) {
      for (int q = threadIdx.x; q < A; q += kBlock) {
        const int gx = x0 + q % AW, gy = y0 + q / AW;
        float v1[3] = {-kShift, -kShift, -kShift}, v2[3] = {-kShift, -kShift, -kShift};  // zero outside
        float vy[3] = {-kShift, -kShift, -kShift};
        if (gx >= 0 && gx < u.width && gy >= 0 && gy < u.height) {
          const float *rp = u.reference + ((int64_t)gy * u.width + gx) * 3;
#pragma unroll
          for (int c = 0; c < 3; ++c) vy[c] = rp[c] - kShift;
          const int nt = (gy / TH) * u.tiles_x + gx / TW;
          if (bit_at(rrow, nt)) {  // outside the region: the same value in both states
            // slot of tile nt within group g's region (the word prefix counts every group)
            const uint32_t w = (uint32_t)nt >> 5, b = (uint32_t)nt & 31u;
            const uint32_t slot = rpre[w] - u.group_base[g] + (uint32_t)__popc(rrow[w] & ((1u << b) - 1u));
            const int64_t it = (int64_t)u.item_base[j] + slot;
            const int lp = (gy - (gy / TH) * TH) * TW + (gx - (gx / TW) * TW);
            const float *pp = u.patches + (it * 2 * kBlock + lp) * 3;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              v1[c] = pp[c] - kShift;
              v2[c] = pp[kBlock * 3 + c] - kShift;
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xs[0][c][q] = v1[c];
          xs[1][c][q] = v2[c];
          ys[c][q] = vy[c];
        }
      }
      __syncthreads();
      const int ox = threadIdx.x % TW, oy = threadIdx.x / TW;
      const bool in = tx * TW + ox < u.width && ty * TH + oy < u.height;
      for (int c = 0; c < 3; ++c) {
        for (int task = threadIdx.x; task < AH * (TW / 2); task += kBlock) {
          const int r = task / (TW / 2), cx = (task % (TW / 2)) * 2;
          const float *ar = &xs[0][c][r * AW + cx], *br = &xs[1][c][r * AW + cx], *yr = &ys[c][r * AW + cx];
          float t0[8], t1[8];
#pragma unroll
          for (int m = 0; m < 8; ++m) t0[m] = t1[m] = 0.0f;
#pragma unroll
          for (int d = 0; d <= 2 * kSsimR + 1; ++d) {
            const float a = ar[d], bb = br[d], y = yr[d];
            const float v[8] = {a, bb, y, a * a, bb * bb, y * y, a * y, bb * y};
            if (d <= 2 * kSsimR) {
#pragma unroll
              for (int m = 0; m < 8; ++m) t0[m] = fmaf(W.w[d], v[m], t0[m]);
            }
            if (d >= 1) {
#pragma unroll
              for (int m = 0; m < 8; ++m) t1[m] = fmaf(W.w[d - 1], v[m], t1[m]);
            }
          }
#pragma unroll
          for (int m = 0; m < 8; ++m) {
            hs[m][r * TW + cx] = t0[m];
            hs[m][r * TW + cx + 1] = t1[m];
          }
        }
        __syncthreads();
        if (in) {
          float mo[8];
#pragma unroll
          for (int m = 0; m < 8; ++m) mo[m] = 0.0f;
#pragma unroll
          for (int d = 0; d <= 2 * kSsimR; ++d) {
            const int q = (oy + d) * TW + ox;
#pragma unroll
            for (int m = 0; m < 8; ++m) mo[m] = fmaf(W.w[d], hs[m][q], mo[m]);
          }
          const int q = (oy + kSsimR) * AW + ox + kSsimR;
          const float d1 = xs[0][c][q] - ys[c][q], d2 = xs[1][c][q] - ys[c][q];
          const float s1 = ssim_value(mo[0], mo[2], mo[3], mo[5], mo[6]);
          const float s2 = ssim_value(mo[1], mo[2], mo[4], mo[5], mo[7]);
          acc += (d1 * d1 - d2 * d2) - u.lambda * (s1 - s2);
        }
        __syncthreads();
      }
    }
    const float tot = block_sum(acc, red);
    if (threadIdx.x == 0) u.partial[item] = tot;
    __syncthreads();
  }
}

// Delta per context: its items' partial sums (in FP64, in item order) / 3HW;
// NaN for an invalid context or after an item overflow.
// Delta per context: its items' sums in a fixed order (one workgroup per
// context, FP64).
__global__ void __launch_bounds__(kBlock)
k_context_delta(UtilArgs u, const uint32_t *__restrict__ bad, float *__restrict__ delta) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const unsigned long long total = *u.item_total;
  if (bad[j] || total > u.item_capacity) {  // uniform over the workgroup
    if (threadIdx.x == 0) delta[j] = __int_as_float(0x7FC00000);
    return;
  }
  const uint32_t b = u.item_base[j], e = j + 1 < u.num_contexts ? u.item_base[j + 1] : (uint32_t)total;
  double s = 0.0;
  for (uint32_t i = b + threadIdx.x; i < e; i += kBlock) s += (double)u.partial[i];
  s = block_sum_f64(s, red);
  if (threadIdx.x == 0) delta[j] = (float)(s / (3.0 * (double)u.width * (double)u.height));
}

// Full images: per (image, 16x16 block) sums of squared error and SSIM.  One
// pass reads the apron of all three channels; the horizontal 11-tap pass of
// the five window sums runs per channel with two output columns per task.
__global__ void __launch_bounds__(kBlock)
k_distortion_tiles(const float *__restrict__ images, const float *__restrict__ reference, int width, int height,
                   int bx, int by, SsimWeights W, double *__restrict__ part) {
  constexpr int AW = 16 + 2 * kSsimR, AH = 16 + 2 * kSsimR, A = AW * AH;
  __shared__ float xs[3][A], ys[3][A];
  __shared__ float hs[5][AH * 16];
  __shared__ float red[4];
  const int blk = blockIdx.x, img = blockIdx.y;
  const int tx = blk % bx, ty = blk / bx;
  const float *im = images + (int64_t)img * width * height * 3;
  const int x0 = tx * 16 - kSsimR, y0 = ty * 16 - kSsimR;
  for (int q = threadIdx.x; q < A; q += kBlock) {
    const int gx = x0 + q % AW, gy = y0 + q / AW;
    float v[3] = {-kShift, -kShift, -kShift}, w[3] = {-kShift, -kShift, -kShift};
    if (gx >= 0 && gx < width && gy >= 0 && gy < height) {
      const int64_t o = ((int64_t)gy * width + gx) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[c] = im[o + c] - kShift;
        w[c] = reference[o + c] - kShift;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xs[c][q] = v[c];
      ys[c][q] = w[c];
    }
  }
  __syncthreads();
  const int ox = threadIdx.x % 16, oy = threadIdx.x / 16;
  const bool in = tx * 16 + ox < width && ty * 16 + oy < height;
  float se = 0.0f, ss = 0.0f;
  for (int c = 0; c < 3; ++c) {
    for (int task = threadIdx.x; task < AH * 8; task += kBlock) {
      const int r = task / 8, cx = (task % 8) * 2;
      const float *xr = &xs[c][r * AW + cx], *yr = &ys[c][r * AW + cx];
      float t0[5], t1[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) t0[m] = t1[m] = 0.0f;
#pragma unroll
      for (int d = 0; d <= 2 * kSsimR + 1; ++d) {
        const float x = xr[d], y = yr[d];
        const float vals[5] = {x, y, x * x, y * y, x * y};
        if (d <= 2 * kSsimR) {
#pragma unroll
          for (int m = 0; m < 5; ++m) t0[m] = fmaf(W.w[d], vals[m], t0[m]);
        }
        if (d >= 1) {
#pragma unroll
          for (int m = 0; m < 5; ++m) t1[m] = fmaf(W.w[d - 1], vals[m], t1[m]);
        }
      }
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        hs[m][r * 16 + cx] = t0[m];
        hs[m][r * 16 + cx + 1] = t1[m];
      }
    }
    __syncthreads();
    if (in) {
      float mo[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int d = 0; d <= 2 * kSsimR; ++d) {
        const int q = (oy + d) * 16 + ox;
#pragma unroll
        for (int m = 0; m < 5; ++m) mo[m] = fmaf(W.w[d], hs[m][q], mo[m]);
      }
      const int q = (oy + kSsimR) * AW + ox + kSsimR;
      const float dv = xs[c][q] - ys[c][q];
      se += dv * dv;
      ss += ssim_value(mo[0], mo[1], mo[2], mo[3], mo[4]);
    }
    __syncthreads();
  }
  const float tse = block_sum(se, red);
  const float tss = block_sum(ss, red);
  if (threadIdx.x == 0) {
    part[((int64_t)img * bx * by + blk) * 2 + 0] = (double)tse;
    part[((int64_t)img * bx * by + blk) * 2 + 1] = (double)tss;
  }
}

// D per image from its blocks' sums (one workgroup per image, fixed order, FP64).
__global__ void __launch_bounds__(kBlock)
k_distortion_finalize(const double *__restrict__ part, int num_images, int blocks, int64_t values, float lambda,
                      float *__restrict__ d) {
  __shared__ double red[4];
  const int img = blockIdx.x;
  double se = 0.0, ss = 0.0;
  for (int b = threadIdx.x; b < blocks; b += kBlock) {
    se += part[((int64_t)img * blocks + b) * 2 + 0];
    ss += part[((int64_t)img * blocks + b) * 2 + 1];
  }
  se = block_sum_f64(se, red);
  ss = block_sum_f64(ss, red);
  if (threadIdx.x == 0) d[img] = (float)(se / (double)values + (double)lambda * (1.0 - ss / (double)values));
}

// ------------------------------------------------------------ Eq. (4)
// One workgroup per group: bitonic sort of its values in LDS, then mean,
// population standard deviation, linear-interpolation quantile (FP64).
__global__ void __launch_bounds__(kBlock)
k_risk_adjusted(const float *__restrict__ values, const int32_t *__restrict__ offsets, float alpha, float beta,
                float q, float *__restrict__ out) {
  __shared__ float v[kMaxRiskValues];
  __shared__ double red[4];
  const int g = blockIdx.x;
  const int b = offsets[g], n = offsets[g + 1] - b;
  float *o = out + (int64_t)g * 4;
  if (n <= 0 || n > kMaxRiskValues) {
    if (threadIdx.x < 4) o[threadIdx.x] = __int_as_float(0x7FC00000);
    return;
  }
  int np = 1;
  while (np < n) np <<= 1;
  bool nan = false;
  for (int i = threadIdx.x; i < np; i += kBlock) {
    const float x = i < n ? values[b + i] : INFINITY;
    v[i] = x;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) nan |= v[i] != v[i];
  if (__syncthreads_or(nan)) {
    if (threadIdx.x < 4) o[threadIdx.x] = __int_as_float(0x7FC00000);
    return;
  }
  for (int k = 2; k <= np; k <<= 1)
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int i = threadIdx.x; i < np; i += kBlock) {
        const int p = i ^ jj;
        if (p > i) {
          const bool up = (i & k) == 0;
          const float a = v[i], c = v[p];
          if ((a > c) == up) {
            v[i] = c;
            v[p] = a;
          }
        }
      }
      __syncthreads();
    }
  // mean and population standard deviation, two passes in FP64
  auto sum = [&](double x) {
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
  };
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += (double)v[i];
  const double mean = sum(s) / n;
  double s2 = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const double d = (double)v[i] - mean;
    s2 += d * d;
  }
  const double sd = sqrt(sum(s2) / n);
  if (threadIdx.x == 0) {
    const double h = (double)(n - 1) * (double)q;
    int lo = (int)floor(h);
    if (lo < 0) lo = 0;
    if (lo > n - 1) lo = n - 1;
    const int hi = lo + 1 < n ? lo + 1 : n - 1;
    const double qv = (double)v[lo] + (h - lo) * ((double)v[hi] - (double)v[lo]);
    o[0] = (float)mean;
    o[1] = (float)qv;
    o[2] = (float)sd;
    o[3] = (float)(((1.0 - alpha) * mean + alpha * qv) / (1.0 + beta * sd));
  }
}

__global__ void k_fill_i32(int *p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_clear_util_header(UtilHeader *h) {
  if (threadIdx.x == 0) *h = UtilHeader{};
}

// ----------------------------------------------------------------- launchers
void launch_clear_util_header(UtilHeader *h, hipStream_t st) { k_clear_util_header<<<1, 64, 0, st>>>(h); }

void launch_group_setup(const UtilArgs &u, const uint16_t *group_pl, int G, int P, const float4 *rec0,
                        const uint2 *rect, int n, int rx, int ry, hipStream_t st) {
  const int64_t gw = (int64_t)G * u.words;
  k_fill_i32<<<(unsigned)std::min<int64_t>(ceil_div((int64_t)P * 4, kBlock), 1024), kBlock, 0, st>>>(u.pl2g, (int64_t)P * 4, -1);
  k_fill_i32<<<(unsigned)std::min<int64_t>(ceil_div(gw, kBlock), 4096), kBlock, 0, st>>>(reinterpret_cast<int *>(u.core), gw, 0);
  k_group_table<<<(unsigned)ceil_div(G, kBlock), kBlock, 0, st>>>(group_pl, G, P, u.pl2g, u.hdr);
  if (n > 0) {
    if (gw <= kCoreLdsWords) {
      const int blocks = (int)std::min<int64_t>(ceil_div(n, kBlock), 128);
      k_group_core<true><<<blocks, kBlock, 0, st>>>(rec0, rect, n, u.pl2g, u.tiles_x, u.words, (int)gw, u.refined,
                                                    u.core);
    } else {
      const int blocks = (int)std::min<int64_t>(ceil_div(n, kBlock), 4096);
      k_group_core<false><<<blocks, kBlock, 0, st>>>(rec0, rect, n, u.pl2g, u.tiles_x, u.words, (int)gw, u.refined,
                                                     u.core);
    }
  }
  k_group_region<<<(unsigned)ceil_div(gw, kBlock), kBlock, 0, st>>>(u.core, G, u.tiles_x, u.tiles_y, u.words,
                                                                    rx, ry, u.region, u.wcount);
  launch_scan_u32(u.wcount, u.wprefix, gw, u.parts, &u.hdr->regions, st);
  k_region_tiles<<<(unsigned)ceil_div(gw, kBlock), kBlock, 0, st>>>(u.region, u.wprefix, gw, u.words,
                                                                    u.region_tiles);
  k_group_base<<<(unsigned)ceil_div(G + 1, kBlock), kBlock, 0, st>>>(u.wprefix, &u.hdr->regions, G, u.words,
                                                                     u.group_base);
}

void launch_pair_setup(const UtilArgs &u, const uint8_t *codes, const uint16_t *group_pl, int G, int P,
                       hipStream_t st) {
  k_pair_setup<<<u.num_contexts, kBlock, 0, st>>>(codes, u.context_group, group_pl, u.group_base, u.num_contexts,
                                                  G, P, u.icount, u.pvis, u.bad, u.hdr, u.refined);
  launch_scan_u32(u.icount, u.item_base, u.num_contexts, u.parts, &u.hdr->items, st);
  k_bundle_setup<<<(unsigned)ceil_div(u.num_contexts, kBlock), kBlock, 0, st>>>(u.context_group, u.bad, u.icount,
                                                                              u.num_contexts, u.bcount);
  launch_scan_u32(u.bcount, u.bbase, u.num_contexts, u.parts, &u.hdr->bundle_items, st);
}

int launch_pair_ssim(const UtilArgs &u, int tile_w, int tile_h, int workgroups, hipStream_t st) {
  const SsimWeights W = ssim_weights();
  launch_zero_queues(u.queue, st);
  if (tile_w == 16 && tile_h == 16)
    k_pair_ssim<16, 16><<<workgroups, kBlock, 0, st>>>(u, W);
  else if (tile_w == 32 && tile_h == 8)
    k_pair_ssim<32, 8><<<workgroups, kBlock, 0, st>>>(u, W);
  else
    return 1;
  k_context_delta<<<(unsigned)u.num_contexts, kBlock, 0, st>>>(u, u.bad, u.delta);
  return 0;
}

void launch_distortion(const float *images, int num_images, int width, int height, const float *reference,
                       float lambda, double *part, float *d, hipStream_t st) {
  const int bx = (int)ceil_div(width, 16), by = (int)ceil_div(height, 16);
  k_distortion_tiles<<<dim3(bx * by, num_images), kBlock, 0, st>>>(images, reference, width, height, bx, by,
                                                                  ssim_weights(), part);
  k_distortion_finalize<<<(unsigned)num_images, kBlock, 0, st>>>(part, num_images, bx * by,
                                                                 (int64_t)width * height * 3, lambda, d);
}

void launch_risk_adjusted(const float *values, const int32_t *offsets, int G, float alpha, float beta, float q,
                          float *out, hipStream_t st) {
  k_risk_adjusted<<<G, kBlock, 0, st>>>(values, offsets, alpha, beta, q, out);
}

}  // namespace dgs
