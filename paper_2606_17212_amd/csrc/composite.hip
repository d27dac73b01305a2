// Masked front-to-back alpha compositing of many delivery states from one set
// of per-tile (depth, index)-sorted lists, forward and backward.
//
// Work item = (tile, group of S states); one 256-thread workgroup, one pixel
// per thread.  The tile's list is walked in batches of 256 entries staged in
// LDS.  The alpha of a splat at a pixel does not depend on the state, so it
// is evaluated once per (pixel, entry) and applied to every state of the
// group that has the entry delivered: the delivery bits of an entry are the
// same for every pixel, so the per-state tests are scalar (wave-uniform)
// branches, and an entry no state of the wave still needs costs four scalar
// instructions.  States are independent recurrences held in registers.
//
// Per (pixel, state): alpha = min(0.99, o exp(-q/2)); alpha < 1/255 is
// skipped; C += T alpha c; T -= T alpha; compositing stops right after the
// entry that leaves T < 1e-4.  A stopped state keeps -T_final in its T slot,
// which makes every later update an exact no-op.  The per-state arithmetic
// is one shared function, so a state's pixels are bit-identical whichever
// group, tile shape or launch they are composited in.
#include "common.h"
#include "kernels.h"

namespace dgs {

__device__ __forceinline__ float splat_alpha_e(float u, float v, float o, float A, float B, float C,
                                               float px, float py, float &e_out) {
  const float dx = u - px, dy = v - py;
  const float q = fmaf(A * dx, dx, fmaf(C * dy, dy, (2.0f * B) * dx * dy));
  const float e = __builtin_amdgcn_exp2f(q * -0.72134752044448170f);  // e^{-q/2}
  e_out = e;
  return fminf(kAlphaMax, o * e);
}

__device__ __forceinline__ void blend(float &T, float &r, float &g, float &b, float alpha, float cr,
                                      float cg, float cb) {
  const float Tp = fmaxf(T, 0.0f);
  const float ta = Tp * alpha;
  r = fmaf(ta, cr, r);
  g = fmaf(ta, cg, g);
  b = fmaf(ta, cb, b);
  const float Tn = T - ta;
  T = (Tn < kTStop) ? -fabsf(Tn) : Tn;
}

// Linear workgroup id -> work item, so that consecutive items land on the
// same XCD (workgroups are dispatched round-robin over the 8 XCDs): the
// groups of one tile and neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_item(int L, int total) {
  const int xcd = L & 7, slot = L >> 3;
  const int q = total >> 3, rm = total & 7;
  return xcd * q + (xcd < rm ? xcd : rm) + slot;
}

template <int S, int TW, int TH, int MODE>
__global__ void __launch_bounds__(kBlock) k_composite(CompositeArgs a) {
  static_assert(TW * TH == kBlock, "one pixel per thread");
  const int total = a.tiles_x * a.tiles_y * a.groups;
  const int item = xcd_item(blockIdx.x, total);
  const int tile = item / a.groups, grp = item - tile * a.groups;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tid = threadIdx.x;
  const int px = tx * TW + (tid % TW), py = ty * TH + (tid / TW);
  const bool inside = px < a.width && py < a.height;
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;

  float T[S], cr[S], cg[S], cb[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    T[s] = inside ? 1.0f : -1.0f;
    cr[s] = cg[s] = cb[s] = 0.0f;
  }

  __shared__ float4 s_a[kBlock];  // u, v, o, delivery bits
  __shared__ float4 s_b[kBlock];  // conic A, B, C, depth
  __shared__ float4 s_c[kBlock];  // colour

  const uint2 rg = a.ranges[tile];
  const uint32_t *vis = a.visbits ? a.visbits + (int64_t)grp * a.P4 : nullptr;
  uint32_t n_alpha = 0, n_blend = 0;  // MODE 2 only
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kBlock) {
    int alive = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) alive |= T[s] > 0.0f;
    if (!__syncthreads_or(alive)) break;
    const uint32_t e = b0 + tid;
    if (e < rg.y) {
      const uint32_t id = a.vals[e];
      const float4 r0 = a.rec0[id];
      const uint32_t vb = vis ? vis[__float_as_uint(r0.w)] : 1u;
      s_a[tid] = make_float4(r0.x, r0.y, r0.z, __uint_as_float(vb));
      s_b[tid] = a.rec1[id];
      s_c[tid] = a.rec2[id];
    }
    __syncthreads();
    uint32_t wave_alive = 0;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (__ballot(T[s] > 0.0f)) wave_alive |= 1u << s;
    const int cnt = (int)((rg.y - b0) < (uint32_t)kBlock ? (rg.y - b0) : (uint32_t)kBlock);
    for (int k = 0; k < cnt; ++k) {
      const float4 A = s_a[k];
      const uint32_t uv = __builtin_amdgcn_readfirstlane(__float_as_uint(A.w)) & wave_alive;
      if (uv == 0u) continue;
      if (MODE == 2) {
        uint32_t lane_alive = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) lane_alive |= (T[s] > 0.0f ? 1u : 0u) << s;
        n_alpha += (uv & lane_alive) ? 1u : 0u;
      }
      const float4 B = s_b[k];
      float e;
      const float alpha = splat_alpha_e(A.x, A.y, A.z, B.x, B.y, B.z, fpx, fpy, e);
      if (alpha < kAlphaMin) continue;
      const float4 C = s_c[k];
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (uv & (1u << s)) {
          if (MODE == 2) n_blend += T[s] > 0.0f ? 1u : 0u;
          blend(T[s], cr[s], cg[s], cb[s], alpha, C.x, C.y, C.z);
        }
    }
    __syncthreads();
  }

  if (MODE == 2) {
    // work counters: alpha evaluations some live delivered state needs, and blends
    unsigned long long c0 = n_alpha, c1 = n_blend;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      c0 += __shfl_xor(c0, d, kWave);
      c1 += __shfl_xor(c1, d, kWave);
    }
    if (__lane_id() == 0) {
      atomicAdd(a.counters, c0);
      atomicAdd(a.counters + 1, c1);
    }
    return;
  }

  if (MODE == 0) {
    if (!inside) return;
    const int64_t pix = (int64_t)py * a.width + px;
    const int64_t plane = (int64_t)a.width * a.height;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int w = a.state_offset + grp * S + s;
      if (w >= a.num_states) break;
      const float Tf = fabsf(T[s]);
      float *o = a.image + ((int64_t)w * plane + pix) * 3;
      o[0] = fmaf(Tf, a.bg[0], cr[s]);
      o[1] = fmaf(Tf, a.bg[1], cg[s]);
      o[2] = fmaf(Tf, a.bg[2], cb[s]);
      if (a.tfinal) a.tfinal[(int64_t)w * plane + pix] = Tf;
    }
  } else {
    // squared error against the reference, reduced over the tile per state
    __shared__ float s_red[4][S];
    float ref[3] = {0.0f, 0.0f, 0.0f};
    if (inside) {
      const float *rp = a.reference + ((int64_t)py * a.width + px) * 3;
      ref[0] = rp[0]; ref[1] = rp[1]; ref[2] = rp[2];
    }
    const int lane = __lane_id(), wv = tid >> 6;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      float se = 0.0f;
      if (inside) {
        const float Tf = fabsf(T[s]);
        const float d0 = fmaf(Tf, a.bg[0], cr[s]) - ref[0];
        const float d1 = fmaf(Tf, a.bg[1], cg[s]) - ref[1];
        const float d2 = fmaf(Tf, a.bg[2], cb[s]) - ref[2];
        se = d0 * d0 + d1 * d1 + d2 * d2;
      }
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) se += __shfl_xor(se, d, kWave);
      if (lane == 0) s_red[wv][s] = se;
    }
    __syncthreads();
    if (tid < S) {
      const int w = a.state_offset + grp * S + tid;
      if (w < a.num_states) {
        const int ntiles = a.tiles_x * a.tiles_y;
        a.psnr_part[(int64_t)w * ntiles + tile] = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_psnr_finalize(const float *__restrict__ part, int tiles, double inv_count, float *__restrict__ psnr) {
  const int w = blockIdx.x;
  double s = 0.0;
  for (int t = threadIdx.x; t < tiles; t += kBlock) s += (double)part[(int64_t)w * tiles + t];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, kWave);
  __shared__ double ws[4];
  if (__lane_id() == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mse = (ws[0] + ws[1] + ws[2] + ws[3]) * inv_count;
    if (mse < 1e-10) mse = 1e-10;
    psnr[w] = (float)(10.0 * log10(1.0 / mse));
  }
}

void launch_psnr_finalize(const float *psnr_part, int num_states, int tiles, int64_t pixels, float *psnr,
                          hipStream_t st) {
  if (num_states <= 0) return;
  k_psnr_finalize<<<num_states, kBlock, 0, st>>>(psnr_part, tiles, 1.0 / (3.0 * (double)pixels), psnr);
}

// ------------------------------------------------------------------ backward

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

// Per tile the forward is replayed front to back with bit-identical
// arithmetic (same alphas, same transmittance updates, same stop), so no
// per-pixel list is stored.  The colour behind entry k comes from the final
// colour minus the running prefix: rem_k = C_final - sum_{j<=k} T_j a_j c_j,
// which includes T_final * background.  Per state and entry:
//   dL/dc_k     = g T_k a_k
//   dL/da_k     = T_k (g . c_k) - (g . rem_k) / (1 - a_k)
// summed over the group's states, then through a = min(0.99, o e^{-q/2}) to
// (u, v, A, B, C, o), reduced over the wave and added to the Gaussian's
// 2D gradient with one atomic per value.
template <int S, int TW, int TH>
__global__ void __launch_bounds__(kBlock) k_composite_bwd(CompositeBwdArgs a) {
  const int total = a.tiles_x * a.tiles_y * a.groups;
  const int item = xcd_item(blockIdx.x, total);
  const int tile = item / a.groups, grp = item - tile * a.groups;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tid = threadIdx.x;
  const int px = tx * TW + (tid % TW), py = ty * TH + (tid / TW);
  const bool inside = px < a.width && py < a.height;
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const int64_t plane = (int64_t)a.width * a.height;
  const int64_t pix = (int64_t)py * a.width + px;

  float T[S], rr[S], rgn[S], rb[S], gr[S], gg[S], gb[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int w = grp * S + s;
    const bool ok = inside && w < a.num_states;
    T[s] = ok ? 1.0f : -1.0f;
    rr[s] = rgn[s] = rb[s] = gr[s] = gg[s] = gb[s] = 0.0f;
    if (ok) {
      const float *im = a.image + ((int64_t)w * plane + pix) * 3;
      const float *gi = a.grad_image + ((int64_t)w * plane + pix) * 3;
      rr[s] = im[0]; rgn[s] = im[1]; rb[s] = im[2];
      gr[s] = gi[0]; gg[s] = gi[1]; gb[s] = gi[2];
    }
  }

  __shared__ float4 s_a[kBlock];
  __shared__ float4 s_b[kBlock];
  __shared__ float4 s_c[kBlock];
  __shared__ uint32_t s_id[kBlock];

  const uint2 rg = a.ranges[tile];
  const uint32_t *vis = a.visbits ? a.visbits + (int64_t)grp * a.P4 : nullptr;
  const int lane = __lane_id();
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kBlock) {
    int alive = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) alive |= T[s] > 0.0f;
    if (!__syncthreads_or(alive)) break;
    const uint32_t e = b0 + tid;
    if (e < rg.y) {
      const uint32_t id = a.vals[e];
      const float4 r0 = a.rec0[id];
      const uint32_t vb = vis ? vis[__float_as_uint(r0.w)] : 1u;
      s_a[tid] = make_float4(r0.x, r0.y, r0.z, __uint_as_float(vb));
      s_b[tid] = a.rec1[id];
      s_c[tid] = a.rec2[id];
      s_id[tid] = id;
    }
    __syncthreads();
    uint32_t wave_alive = 0;
#pragma unroll
    for (int s = 0; s < S; ++s)
      if (__ballot(T[s] > 0.0f)) wave_alive |= 1u << s;
    const int cnt = (int)((rg.y - b0) < (uint32_t)kBlock ? (rg.y - b0) : (uint32_t)kBlock);
    for (int k = 0; k < cnt; ++k) {
      const float4 A = s_a[k];
      const uint32_t uv = __builtin_amdgcn_readfirstlane(__float_as_uint(A.w)) & wave_alive;
      if (uv == 0u) continue;
      const float4 B = s_b[k];
      float ev;
      const float alpha = splat_alpha_e(A.x, A.y, A.z, B.x, B.y, B.z, fpx, fpy, ev);
      const bool hit = alpha >= kAlphaMin;
      if (!__ballot(hit)) continue;
      float d_alpha = 0.0f, dcr = 0.0f, dcg = 0.0f, dcb = 0.0f;
      float gu = 0.0f, gv = 0.0f, gA = 0.0f, gB = 0.0f, gC = 0.0f, go = 0.0f;
      if (hit) {
        const float4 C = s_c[k];
        const float inv1ma = 1.0f / (1.0f - alpha);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          if (uv & (1u << s)) {
            const float Tp = fmaxf(T[s], 0.0f);
            const float ta = Tp * alpha;
            rr[s] = fmaf(-ta, C.x, rr[s]);
            rgn[s] = fmaf(-ta, C.y, rgn[s]);
            rb[s] = fmaf(-ta, C.z, rb[s]);
            const float gcol = gr[s] * C.x + gg[s] * C.y + gb[s] * C.z;
            const float grem = gr[s] * rr[s] + gg[s] * rgn[s] + gb[s] * rb[s];
            const float da = Tp * gcol - grem * inv1ma;
            d_alpha += (Tp > 0.0f) ? da : 0.0f;
            dcr = fmaf(gr[s], ta, dcr);
            dcg = fmaf(gg[s], ta, dcg);
            dcb = fmaf(gb[s], ta, dcb);
            const float Tn = T[s] - ta;
            T[s] = (Tn < kTStop) ? -fabsf(Tn) : Tn;
          }
        }
        // alpha = o e when below the cap; the cap passes no gradient
        if (A.z * ev < kAlphaMax) {
          const float dpow = d_alpha * alpha;  // d alpha / d power = alpha
          go = d_alpha * ev;
          const float dx = A.x - fpx, dy = A.y - fpy;
          gu = -dpow * (B.x * dx + B.y * dy);
          gv = -dpow * (B.y * dx + B.z * dy);
          gA = -0.5f * dpow * dx * dx;
          gB = -dpow * dx * dy;
          gC = -0.5f * dpow * dy * dy;
        }
      }
      gu = wave_sum(gu); gv = wave_sum(gv); gA = wave_sum(gA); gB = wave_sum(gB); gC = wave_sum(gC);
      go = wave_sum(go); dcr = wave_sum(dcr); dcg = wave_sum(dcg); dcb = wave_sum(dcb);
      if (lane == 0) {
        const uint32_t id = s_id[k];
        float *g = a.g2d;
        const int64_t n = a.n;
        unsafeAtomicAdd(g + id, gu);
        unsafeAtomicAdd(g + n + id, gv);
        unsafeAtomicAdd(g + 2 * n + id, gA);
        unsafeAtomicAdd(g + 3 * n + id, gB);
        unsafeAtomicAdd(g + 4 * n + id, gC);
        unsafeAtomicAdd(g + 5 * n + id, go);
        unsafeAtomicAdd(g + 6 * n + id, dcr);
        unsafeAtomicAdd(g + 7 * n + id, dcg);
        unsafeAtomicAdd(g + 8 * n + id, dcb);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launchers

template <int S, int TW, int TH>
static void launch_fwd_t(const CompositeArgs &a, int mode, unsigned blocks, hipStream_t st) {
  if (mode == 0)
    k_composite<S, TW, TH, 0><<<blocks, kBlock, 0, st>>>(a);
  else if (mode == 1)
    k_composite<S, TW, TH, 1><<<blocks, kBlock, 0, st>>>(a);
  else
    k_composite<S, TW, TH, 2><<<blocks, kBlock, 0, st>>>(a);
}

template <int TW, int TH>
static int launch_fwd_s(const CompositeArgs &a, int S, int mode, unsigned blocks, hipStream_t st) {
  switch (S) {
    case 1: launch_fwd_t<1, TW, TH>(a, mode, blocks, st); return 0;
    case 2: launch_fwd_t<2, TW, TH>(a, mode, blocks, st); return 0;
    case 4: launch_fwd_t<4, TW, TH>(a, mode, blocks, st); return 0;
    case 8: launch_fwd_t<8, TW, TH>(a, mode, blocks, st); return 0;
    case 16: launch_fwd_t<16, TW, TH>(a, mode, blocks, st); return 0;
    case 32: launch_fwd_t<32, TW, TH>(a, mode, blocks, st); return 0;
    default: return 1;
  }
}

int launch_composite(const CompositeArgs &a, int S, int tile_w, int tile_h, int mode, hipStream_t st) {
  const int64_t total = (int64_t)a.tiles_x * a.tiles_y * a.groups;
  if (total <= 0) return 0;
  const unsigned blocks = (unsigned)total;
  if (tile_w == 16 && tile_h == 16) return launch_fwd_s<16, 16>(a, S, mode, blocks, st);
  if (tile_w == 32 && tile_h == 8) return launch_fwd_s<32, 8>(a, S, mode, blocks, st);
  return 1;
}

template <int TW, int TH>
static int launch_bwd_s(const CompositeBwdArgs &a, int S, unsigned blocks, hipStream_t st) {
  switch (S) {
    case 1: k_composite_bwd<1, TW, TH><<<blocks, kBlock, 0, st>>>(a); return 0;
    case 2: k_composite_bwd<2, TW, TH><<<blocks, kBlock, 0, st>>>(a); return 0;
    case 4: k_composite_bwd<4, TW, TH><<<blocks, kBlock, 0, st>>>(a); return 0;
    case 8: k_composite_bwd<8, TW, TH><<<blocks, kBlock, 0, st>>>(a); return 0;
    default: return 1;
  }
}

int launch_composite_bwd(const CompositeBwdArgs &a, int S, int tile_w, int tile_h, hipStream_t st) {
  const int64_t total = (int64_t)a.tiles_x * a.tiles_y * a.groups;
  if (total <= 0) return 0;
  const unsigned blocks = (unsigned)total;
  if (tile_w == 16 && tile_h == 16) return launch_bwd_s<16, 16>(a, S, blocks, st);
  if (tile_w == 32 && tile_h == 8) return launch_bwd_s<32, 8>(a, S, blocks, st);
  return 1;
}

}  // namespace dgs
