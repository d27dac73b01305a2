// Masked front-to-back alpha compositing of many delivery states from one set
// of per-tile (depth, index)-sorted lists, forward and backward.
//
// Work item = (tile, group of S states); one 256-thread workgroup, one pixel
// per thread, each wave owning an 8x8 pixel block of the tile.  The tile's
// list is walked in batches of 256 entries staged in LDS; the thread that
// stages an entry also records, per wave, whether the entry's pixel rectangle
// touches that wave's block and which of the group's states have the entry
// delivered (one 32-bit word per wave).  The alpha of a splat at a pixel
// does not depend on the state, so it is evaluated once per (pixel, entry) and
// applied to every state of the group that has the entry delivered.  The
// delivery word is wave-uniform, so the per-state tests are scalar branches,
// and an entry no live state of the wave needs costs one LDS read and a few
// scalar instructions.
//
// Per (pixel, state): alpha = min(0.99, o exp(-q/2)), evaluated as
// 2^(q' + log2 o) with a pre-scaled conic; alpha < 1/255 is skipped (tested
// on the exponent, before the exponential); C += T alpha c; T -= T alpha;
// compositing stops right after the entry that leaves T < 1e-4.  A stopped
// state keeps -T_final in its T slot; the clamped product clamp(T alpha)
// then makes every later update an exact no-op.  The per-state arithmetic is
// one shared function, so a state's pixels are bit-identical whichever
// group, tile shape or launch they are composited in.
#include "common.h"
#include "kernels.h"

namespace dgs {

// q' = A' dx^2 + B' dx dy + C' dy^2 + log2(o) for p0 = (u, v, log2 o, A'), p1 = (B', C')
__device__ __forceinline__ float splat_q(const float4 &p0, const float2 &p1, float px, float py) {
  const float dx = p0.x - px, dy = p0.y - py;
  float t = p0.w * dx;
  t = fmaf(p1.x, dy, t);
  const float q = fmaf(t, dx, p0.z);
  const float c = p1.y * dy;
  return fmaf(c, dy, q);
}

__device__ __forceinline__ float alpha_of(float q) {
  return fminf(kAlphaMax, __builtin_amdgcn_exp2f(q));
}

__device__ __forceinline__ void blend(float &T, float &r, float &g, float &b, float alpha, float cr,
                                      float cg, float cb) {
  // T alpha for a live state (T > 0, T alpha < 1), exactly 0 for a stopped one (T <= 0)
  const float ta = __builtin_amdgcn_fmed3f(T * alpha, 0.0f, 1.0f);
  r = fmaf(ta, cr, r);
  g = fmaf(ta, cg, g);
  b = fmaf(ta, cb, b);
  const float Tn = T - ta;
  T = (Tn < kTStop) ? -fabsf(Tn) : Tn;
}

// Workgroup id -> (position in the tile order, state group).  Workgroups are
// dispatched in id order, round-robin over the 8 XCDs; the mapping keeps all
// groups of a tile on one XCD (sharing its L2) and starts the heaviest tiles
// first.  Returns false for the idle workgroups of the last row.
__device__ __forceinline__ bool work_item(int L, int groups, int tiles, int &k, int &grp) {
  const int xcd = L & 7, r = L >> 3;
  grp = r % groups;
  k = (r / groups) * 8 + xcd;
  return k < tiles;
}

__host__ __device__ inline int work_items(int tiles, int groups) { return ((tiles + 7) / 8) * 8 * groups; }


struct StageRec {
  float4 p0;   // u, v, log2 o, A'
  float2 p1;   // B', C'
  float2 pad;
  float4 col;  // r, g, b, -
};

// A copy of an LDS pointer that the compiler must keep in a vector register
// (reads through it stay LDS reads).
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using lds_cptr = const __attribute__((address_space(3))) T *;

template <typename T>
__device__ __forceinline__ lds_cptr<T> vgpr_lds_ptr(const T *p) {
  uint32_t a = (uint32_t)(uintptr_t)(lds_cptr<T>)p;
  asm volatile("v_mov_b32 %0, %1" : "=v"(a) : "s"(a));
  return (lds_cptr<T>)(uintptr_t)a;
}
#else  // the host pass only parses device code
template <typename T>
__device__ __forceinline__ const T *vgpr_lds_ptr(const T *p) { return p; }
#endif

// One LDS batch of B list entries.
template <int B>
struct StageT {
  uint32_t vis[4][B];  // per wave: delivery bits of the entry, 0 if it misses the wave's block
  StageRec rec[B];     // one 48-byte record per entry: one LDS base address per entry
  uint32_t id[B];      // Gaussian id (backward)
};
using Stage = StageT<kBlock>;

// Stages one list entry.  The sorted value carries the Gaussian id in its low
// 28 bits and, in bits 28..31, whether the entry can reach alpha >= 1/255 in
// each of the tile's four 8x8 wave blocks (decided once at emission).  Per wave
// the stage holds the entry's delivery bits, or 0 for a block it cannot reach.
// In pair mode `nvis` contexts' two-bit tables, `vstride` words apart, are
// merged: bits 2c and 2c + 1 belong to the bundle's context c.
template <int TW, int TH, typename ST>
__device__ __forceinline__ void stage_entry(ST &st, int slot, uint32_t val, const float4 *rec0,
                                            const float4 *rec1, const float4 *rec2, const uint32_t *vis,
                                            int nvis = 1, int64_t vstride = 0) {
  const uint32_t id = val & kIdMask;
  const float4 r0 = rec0[id];
  const float4 r1 = rec1[id];
  const uint32_t pl = __float_as_uint(r0.w);
  uint32_t vb = vis ? vis[pl] : 1u;
  for (int c = 1; c < nvis; ++c) vb |= vis[c * vstride + pl] << (2 * c);
#pragma unroll
  for (int w = 0; w < 4; ++w) st.vis[w][slot] = ((val >> (kMaskShift + w)) & 1u) ? vb : 0u;
  st.rec[slot].p0 = make_float4(r0.x, r0.y, r0.z, r1.x);
  st.rec[slot].p1 = make_float2(r1.y, r1.z);
  st.rec[slot].col = rec2[id];
  st.id[slot] = id;
}

// Occupancy requested from the register allocator: the state registers
// (4 per state) dominate, so small groups can keep 8 waves per SIMD; 16
// states ask for 6 (80 registers: a few per-item values then live in scratch
// outside the entry loop, which costs less than the sixth wave gains); a
// 512-entry LDS batch (~35 KB) leaves room for 4 workgroups per CU.
template <int S, int B = kBlock>
constexpr int waves_per_eu() {
  constexpr int by_regs = S <= 8 ? 8 : (S <= 16 ? 6 : 2);
  constexpr int by_lds = B > kBlock ? 4 : 8;
  return by_regs < by_lds ? by_regs : by_lds;
}

// Pair mode: a bundle of contexts (their delivery tables `vstride` words
// apart from `vis`) and the work item of each context's patch.
struct PairOut {
  int pairs;
  int64_t vstride;
  uint32_t item[4];
};

// Composites one tile for the S states of one group.  `vis` holds the
// group's delivery bits per (packet, layer); `grp` indexes the outputs (the
// state group); in pair mode `po` names the bundle's patches instead.
template <int S, int TW, int TH, int MODE, int B = kBlock>
__device__ __forceinline__ void composite_item(const CompositeArgs &a, StageT<B> &st, int tile, int grp,
                                               const uint32_t *vis, const PairOut *po = nullptr) {
  static_assert(TW * TH == kBlock, "one pixel per thread");
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int tpx = tx * TW, tpy = ty * TH;
  const int px = tpx + wave_block_x0(wv, TW) + (lane & 7), py = tpy + wave_block_y0(wv, TW) + (lane >> 3);
  const bool inside = px < a.width && py < a.height;
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;

  float T[S], cr[S], cg[S], cb[S];
  const int nact = MODE == 3 ? 2 * po->pairs : S;  // states of the bundle's contexts
#pragma unroll
  for (int s = 0; s < S; ++s) {
    T[s] = (inside && s < nact) ? 1.0f : -1.0f;
    cr[s] = cg[s] = cb[s] = 0.0f;
  }

  const uint2 rg = a.ranges[tile];
  uint32_t n_alpha = 0, n_blend = 0, n_wave_alpha = 0, n_wave_miss = 0;  // MODE 2 only
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += B) {
    int alive = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) alive |= T[s] > 0.0f;
    if (!__syncthreads_or(alive)) break;
#pragma unroll
    for (int off = tid; off < B; off += kBlock) {
      const uint32_t e = b0 + off;
      if (e < rg.y) {
        if (MODE == 3)
          stage_entry<TW, TH>(st, off, a.vals[e], a.rec0, a.rec1, a.rec2, vis, po->pairs, po->vstride);
        else
          stage_entry<TW, TH>(st, off, a.vals[e], a.rec0, a.rec1, a.rec2, vis);
      }
    }
    __syncthreads();
    // entries of this batch; wave-uniform, kept in scalar registers
    const int cnt = __builtin_amdgcn_readfirstlane(
        (int)((rg.y - b0) < (uint32_t)B ? (rg.y - b0) : (uint32_t)B));
    uint32_t wave_alive = 0;
    // four entries per step: one 16-byte read of their delivery bits and
    // constant offsets from one record address
    for (int k0 = 0; k0 < cnt; k0 += 4) {
      if ((k0 & 63) == 0) {  // states still compositing some pixel of this wave
        wave_alive = 0;
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (__ballot(T[s] > 0.0f)) wave_alive |= 1u << s;
      }
      const uint4 v4 = *reinterpret_cast<const uint4 *>(&st.vis[wv][k0]);
      const uint32_t vv[4] = {v4.x, v4.y, v4.z, v4.w};
      // The record address is wave-uniform; held in a vector register (one
      // move per four entries) the reads below use it with immediate offsets
      // instead of a move from a scalar register before every read.
      const StageRec *rp = vgpr_lds_ptr(&st.rec[k0]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (k0 + j >= cnt) break;
        const uint32_t uv = __builtin_amdgcn_readfirstlane(vv[j]) & wave_alive;
        if (uv == 0u) continue;
        if (MODE == 2) {
          uint32_t lane_alive = 0;
#pragma unroll
          for (int s = 0; s < S; ++s) lane_alive |= (T[s] > 0.0f ? 1u : 0u) << s;
          n_alpha += (uv & lane_alive) ? 1u : 0u;
        }
        const float4 P0 = rp[j].p0;
        const float2 P1 = rp[j].p1;
        const float q = splat_q(P0, P1, fpx, fpy);
        if (MODE == 2) {  // every lane is active here: the ballot sees the whole wave
          const bool none = __ballot(q >= kQSkip) == 0ull;
          if (lane == 0) {
            ++n_wave_alpha;
            n_wave_miss += none ? 1u : 0u;
          }
        }
        if (q < kQSkip) continue;
        const float alpha = alpha_of(q);
        const float4 C = rp[j].col;
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (uv & (1u << s)) {
            if (MODE == 2) n_blend += T[s] > 0.0f ? 1u : 0u;
            blend(T[s], cr[s], cg[s], cb[s], alpha, C.x, C.y, C.z);
          }
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
      atomicAdd(a.counters + 2, (unsigned long long)n_wave_alpha);
      atomicAdd(a.counters + 3, (unsigned long long)n_wave_miss);
    }
    return;
  }

  if (MODE == 3) {
    // pair mode: the tile's pixels of both states of each context into that
    // context's work-item patch [item][2][TW * TH][3]
    if (!inside) return;
    const int64_t pix = (int64_t)(py - tpy) * TW + (px - tpx);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (s >= nact) break;
      const float Tf = fabsf(T[s]);
      float *o = a.image + (((int64_t)po->item[s >> 1] * 2 + (s & 1)) * kBlock + pix) * 3;
      o[0] = fmaf(Tf, a.bg[0], cr[s]);
      o[1] = fmaf(Tf, a.bg[1], cg[s]);
      o[2] = fmaf(Tf, a.bg[2], cb[s]);
    }
    return;
  }

  if (MODE == 0) {
    if (!inside) return;
    const int64_t pix = (int64_t)py * a.width + px;
    const int64_t plane = (int64_t)a.width * a.height;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int slot = grp * S + s;
      if (slot >= a.launch_states) break;
      const int w = a.state_offset + (a.state_order ? (int)a.state_order[slot] : slot);
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
    if (tid < S && grp * S + tid < a.launch_states) {
      const int slot = grp * S + tid;
      const int w = a.state_offset + (a.state_order ? (int)a.state_order[slot] : slot);
      {
        const int ntiles = a.tiles_x * a.tiles_y;
        a.psnr_part[(int64_t)w * ntiles + tile] = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
      }
    }
  }
}

// Grid launch: one workgroup per work item (see work_item).  Persistent
// launch: one workgroup per resident slot; each drains its XCD's queue of
// work items in the same heavy-first order, then steals from the other XCDs'
// queues.  Every workgroup leaves once all eight queues are exhausted.
template <int S, int TW, int TH, int MODE, bool PERSISTENT, int B = kBlock>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(waves_per_eu<S, B>(), 8)))
k_composite(CompositeArgs a) {
  __shared__ StageT<B> st;
  const int tiles = a.tiles_x * a.tiles_y;
  int kpos, grp;
  if (!PERSISTENT) {
    if (work_item(blockIdx.x, a.groups, tiles, kpos, grp))
      composite_item<S, TW, TH, MODE, B>(a, st, (int)a.tile_order[kpos], grp,
                                      a.visbits ? a.visbits + (int64_t)grp * a.P4 : nullptr);
    return;
  }
  __shared__ int s_item;
  const int home = blockIdx.x & 7;
  int q = 0;  // queues tried so far (thread 0)
  for (;;) {
    if (threadIdx.x == 0) {
      int item = -1;
      while (q < 8) {
        const int x = (home + q) & 7;
        const int L = (int)atomicAdd(&a.queues[x], 1u) * 8 + x;
        int kk, gg;
        if (work_item(L, a.groups, tiles, kk, gg)) {
          item = L;
          break;
        }
        ++q;  // queue x is exhausted: its later items are further out still
      }
      s_item = item;
    }
    __syncthreads();
    const int L = s_item;
    __syncthreads();
    if (L < 0) break;
    work_item(L, a.groups, tiles, kpos, grp);
    composite_item<S, TW, TH, MODE, B>(a, st, (int)a.tile_order[kpos], grp,
                                    a.visbits ? a.visbits + (int64_t)grp * a.P4 : nullptr);
    __syncthreads();  // the stage is reused by the next item
  }
}

// Paired states of the counterfactual utility.  Each context j has one work
// item per tile of its group's region; the states of a pair (the context m
// and m u g) differ only in g.  Up to four consecutive contexts of one group
// (a bundle) are composited together at one tile as one 8-state group, so
// each splat's alpha serves all eight states; every context's two states go
// to its own item's patch.  Resident workgroups take (bundle, region tile)
// items from one queue.
template <int TW, int TH>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_composite_pairs(CompositeArgs a) {
  __shared__ Stage st;
  __shared__ int s_item;
  // after an overflow nothing is composited (every delta becomes NaN)
  const bool over = *a.pair.item_total > a.pair.item_capacity;
  const unsigned long long total = *a.pair.bundle_total;
  const uint32_t n_items = over ? 0u : (uint32_t)total;
  const int J = a.pair.num_contexts;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(a.queues, 1u);
    __syncthreads();
    const uint32_t item = (uint32_t)s_item;
    __syncthreads();
    if (item >= n_items) break;
    // bundle of the item: the last context b with bundle_base[b] <= item
    int lo = 0, hi = J - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.pair.bundle_base[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const int b = lo;
    const int g = a.pair.context_group[b];
    const uint32_t slot = item - a.pair.bundle_base[b];
    PairOut po;
    po.pairs = 1;
    while (po.pairs < 4 && b + po.pairs < J && !bundle_start(a.pair.context_group, a.pair.bad, b + po.pairs))
      ++po.pairs;
    po.vstride = a.P4;
#pragma unroll
    for (int c = 0; c < 4; ++c) po.item[c] = c < po.pairs ? a.pair.item_base[b + c] + slot : 0u;
    const int tile = (int)a.pair.region_tiles[a.pair.group_base[g] + slot];
    composite_item<8, TW, TH, 3>(a, st, tile, 0, a.visbits + (int64_t)b * a.P4, &po);
    __syncthreads();
  }
}

int launch_composite_pairs(const CompositeArgs &a, int tile_w, int tile_h, int workgroups, hipStream_t st) {
  if (workgroups <= 0) return 0;
  launch_zero_queues(a.queues, st);
  if (tile_w == 16 && tile_h == 16)
    k_composite_pairs<16, 16><<<workgroups, kBlock, 0, st>>>(a);
  else if (tile_w == 32 && tile_h == 8)
    k_composite_pairs<32, 8><<<workgroups, kBlock, 0, st>>>(a);
  else
    return 1;
  return 0;
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

// One DPP step of a row scan: x plus the value CTRL moves into this lane
// (zero where the source lies outside the row).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_step(float x) {
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, true);
  return x + __int_as_float(y);
}

// Two values folded over the wave halves into one register: lanes 0-31 hold
// x[i] + x[i+32], lanes 32-63 hold y[i-32] + y[i] (one half swap, one add).
__device__ __forceinline__ float half_pair_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// Two half-folded registers folded over row pairs into one: row 0 holds the
// sum of x's rows 0-1, row 1 of y's rows 0-1, row 2 of x's rows 2-3, row 3
// of y's rows 2-3.
__device__ __forceinline__ float row_pair_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// Inclusive scan within each 16-lane row: lane 15 of a row holds its sum.
__device__ __forceinline__ float row_sum_to_lane15(float x) {
  x = dpp_step<0x111, 0xf>(x);  // row_shr:1
  x = dpp_step<0x112, 0xf>(x);  // row_shr:2
  x = dpp_step<0x114, 0xf>(x);  // row_shr:4
  x = dpp_step<0x118, 0xf>(x);  // row_shr:8
  return x;
}

// Per tile the forward is replayed front to back with bit-identical
// arithmetic (same alphas, same transmittance updates, same stop), so no
// per-pixel list is stored.  The colour behind entry k is the final colour
// minus the running prefix, rem_k = C_final - sum_{j<=k} T_j a_j c_j (which
// includes T_final * background); only its dot product with g = dL/dC enters,
// so each state keeps the scalar g . rem_k, starting from g . C_final and
// lowered by T_k a_k (g . c_k) at each entry.  Per state and entry:
//   dL/dc_k     = g T_k a_k
//   dL/da_k     = T_k (g . c_k) - (g . rem_k) / (1 - a_k)
// summed over the group's states; then, below the 0.99 cap, through
// a = 2^q' to (u, v, A', B', C', log2 o), reduced over the wave with lane
// swaps and DPP, stored per wave in LDS for a window of 64 entries, folded over the four
// waves and added to the Gaussian's 2D gradient with one atomic per value
// and entry.
constexpr int kBwdWindow = 64;  // entries per fold of the backward's per-wave gradient sums
constexpr int kBwdVals = 9;     // nine values per entry
// Six waves per SIMD: the stage (17 KB) and the window sums (9 KB) let six
// workgroups share a CU's 160 KB of LDS, and at most 80 VGPRs fit six waves.

template <int S, int TW, int TH>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_composite_bwd(CompositeBwdArgs a) {
  int kpos, grp;
  if (!work_item(blockIdx.x, a.groups, a.tiles_x * a.tiles_y, kpos, grp)) return;
  const int tile = (int)a.tile_order[kpos];
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int tpx = tx * TW, tpy = ty * TH;
  const int px = tpx + wave_block_x0(wv, TW) + (lane & 7), py = tpy + wave_block_y0(wv, TW) + (lane >> 3);
  const bool inside = px < a.width && py < a.height;
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
  const int64_t plane = (int64_t)a.width * a.height;
  const int64_t pix = (int64_t)py * a.width + px;

  // per state: transmittance, dL/dC, and g . rem (the colour still to come
  // behind the current entry, dotted with dL/dC) as one scalar
  float T[S], grem[S], gr[S], gg[S], gb[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int slot = grp * S + s;
    const bool ok = inside && slot < a.num_states;
    const int w = ok ? (a.state_order ? (int)a.state_order[slot] : slot) : 0;
    T[s] = ok ? 1.0f : -1.0f;
    grem[s] = gr[s] = gg[s] = gb[s] = 0.0f;
    if (ok) {
      const float *im = a.image + ((int64_t)w * plane + pix) * 3;
      const float *gi = a.grad_image + ((int64_t)w * plane + pix) * 3;
      gr[s] = gi[0]; gg[s] = gi[1]; gb[s] = gi[2];
      grem[s] = fmaf(gr[s], im[0], fmaf(gg[s], im[1], gb[s] * im[2]));
    }
  }

  __shared__ Stage st;
  // per-entry gradient sums of each wave over a window of kBwdWindow entries:
  // [wave][entry][value] (plain stores, folded once per window)
  __shared__ float red[4][kBwdWindow][kBwdVals];
  const uint2 rg = a.ranges[tile];
  const uint32_t *vis = a.visbits ? a.visbits + (int64_t)grp * a.P4 : nullptr;
  float *red_flat = &red[0][0][0];
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kBlock) {
    int alive = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) alive |= T[s] > 0.0f;
    if (!__syncthreads_or(alive)) break;
    const uint32_t e = b0 + tid;
    if (e < rg.y) stage_entry<TW, TH>(st, tid, a.vals[e], a.rec0, a.rec1, a.rec2, vis);
    const int cnt = (int)((rg.y - b0) < (uint32_t)kBlock ? (rg.y - b0) : (uint32_t)kBlock);
    for (int w0 = 0; w0 < cnt; w0 += kBwdWindow) {
      for (int i = tid; i < 4 * kBwdWindow * kBwdVals; i += kBlock) red_flat[i] = 0.0f;
      __syncthreads();  // stage (first window) and cleared sums visible
      const int w1 = (w0 + kBwdWindow) < cnt ? (w0 + kBwdWindow) : cnt;
      uint32_t wave_alive = 0;
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (__ballot(T[s] > 0.0f)) wave_alive |= 1u << s;
      for (int k = w0; k < w1; ++k) {
        const uint32_t uv = __builtin_amdgcn_readfirstlane(st.vis[wv][k]) & wave_alive;
        if (uv == 0u) continue;
        const float4 P0 = st.rec[k].p0;
        const float2 P1 = st.rec[k].p1;
        const float q = splat_q(P0, P1, fpx, fpy);
        const bool hit = q >= kQSkip;
        if (!__ballot(hit)) continue;
        // A lane the splat misses (alpha < 1/255) takes alpha = 0 instead of a
        // branch: then T alpha = 0, every update below leaves T, g . rem and
        // the colour sums exactly as they are (a live T is >= the stop bound),
        // and dq = d_alpha x 0 makes every gradient term zero.
        const float alpha = hit ? alpha_of(q) : 0.0f;
        const float4 C = st.rec[k].col;
        // hardware reciprocal (about 1 ulp; 1 - alpha >= 0.01 under the cap)
        // instead of the IEEE division sequence
        const float inv1ma = __builtin_amdgcn_rcpf(1.0f - alpha);
        // dL/dalpha = sum over the delivered states of T g . c - (g . rem_k) / (1 - alpha),
        // kept as the two sums (the second scaled once per entry)
        float dcr = 0.0f, dcg = 0.0f, dcb = 0.0f, sum_tg = 0.0f, sum_rem = 0.0f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          if (uv & (1u << s)) {
            const float ta = __builtin_amdgcn_fmed3f(T[s] * alpha, 0.0f, 1.0f);
            const float gcol = fmaf(gr[s], C.x, fmaf(gg[s], C.y, gb[s] * C.z));
            grem[s] = fmaf(-ta, gcol, grem[s]);  // g . rem_k
            // zero for a stopped state (T and g . rem both cleared at the stop)
            // and for a lane outside the image (T = -1, g = 0)
            sum_tg = fmaf(T[s], gcol, sum_tg);
            sum_rem += grem[s];
            dcr = fmaf(gr[s], ta, dcr);
            dcg = fmaf(gg[s], ta, dcg);
            dcb = fmaf(gb[s], ta, dcb);
            const float Tn = T[s] - ta;
            const bool stop = Tn < kTStop;
            // the replay needs T only for T alpha (zero once stopped, as in
            // the forward's -T_final) and the liveness tests
            T[s] = stop ? 0.0f : Tn;
            grem[s] = stop ? 0.0f : grem[s];
          }
        }
        // below the cap alpha = 2^q': d alpha / d q' = alpha ln 2; the cap
        // passes nothing.  dq'/du = 2 A' dx + B' dy and dq'/dv = B' dx + 2 C' dy
        // are linear in (dx, dy) with entry constants, so the lanes sum
        // dq dx and dq dy (in the gu, gv slots) and the fold applies A', B', C'.
        const float d_alpha = fmaf(-sum_rem, inv1ma, sum_tg);
        const float dq = alpha < kAlphaMax ? d_alpha * alpha * 0.69314718055994531f : 0.0f;
        const float dx = P0.x - fpx, dy = P0.y - fpy;
        const float gu = dq * dx, gv = dq * dy;
        const float gA = gu * dx, gB = gu * dy, gC = gv * dy, glo = dq;
        // the nine wave sums share their steps: halves, then row pairs fold
        // values into registers that hold four (one per row), then row scans;
        // register q0 ends with rows (gu, gA, gv, gB), q1 with (gC, dcr, glo,
        // dcg), q2 with dcb in every row
        const float q0 = row_sum_to_lane15(row_pair_sum(half_pair_sum(gu, gv), half_pair_sum(gA, gB)));
        const float q1 = row_sum_to_lane15(row_pair_sum(half_pair_sum(gC, glo), half_pair_sum(dcr, dcg)));
        const float d8 = half_pair_sum(dcb, dcb);
        const float q2 = row_sum_to_lane15(row_pair_sum(d8, d8));
        if ((lane & 15) == 15) {  // this wave's sums for entry k: plain LDS stores
          const int row = lane >> 4, v = ((row & 1) << 1) | (row >> 1);
          float *o = red[wv][k - w0];
          o[v] = q0;
          o[4 + v] = q1;
          if (row == 0) o[8] = q2;
        }
      }
      __syncthreads();
      // fold the four waves; one atomic per value and entry for the workgroup
      // (values 0 and 1 from the sums of dq dx and dq dy)
      for (int i = tid; i < (w1 - w0) * 9; i += kBlock) {
        const int k = i / 9, v = i - k * 9;
        float sum = red[0][k][v] + red[1][k][v] + red[2][k][v] + red[3][k][v];
        if (v < 2) {
          const int o = v ^ 1;
          const float other = red[0][k][o] + red[1][k][o] + red[2][k][o] + red[3][k][o];
          const StageRec &r = st.rec[w0 + k];
          // v = 0: 2 A' Sx + B' Sy;  v = 1: B' Sx + 2 C' Sy
          sum = v == 0 ? fmaf(2.0f * r.p0.w, sum, r.p1.x * other) : fmaf(r.p1.x, other, 2.0f * r.p1.y * sum);
        }
        if (sum != 0.0f) unsafeAtomicAdd(a.g2d + (int64_t)v * a.n + st.id[w0 + k], sum);
      }
      __syncthreads();  // sums read before the next window clears them
    }
  }
}

// ------------------------------------------------------------------ launchers

// Automatic choice: the persistent launch pays off once the grid would hold
// many waves of workgroups (per-workgroup launch cost dominates the saving),
// and for groups of 16 or more states (long work items) from a few items per
// resident workgroup on.
constexpr int kPersistentItemsPerSlot = 32;
constexpr int kPersistentMinStates = 16;
constexpr int kPersistentItemsPerSlotLarge = 4;

// Resident workgroups of the persistent kernel, cached per instantiation
// (host-side queries only, so a launch can be captured in a graph).
template <int S, int TW, int TH, int MODE, int B>
static int resident_slots() {
  static int resident = 0;
  if (!resident) {
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_composite<S, TW, TH, MODE, true, B>, kBlock, 0);
    resident = (cus > 0 ? cus : 256) * (per_cu > 0 ? per_cu : 1);
  }
  return resident;
}

template <int S, int TW, int TH, int MODE, int B>
static CompositePlan plan_fwd_m(int launch, int64_t items) {
  const int64_t resident = resident_slots<S, TW, TH, MODE, B>();
  CompositePlan p;
  p.items = items;
  p.persistent = launch == 1 || (launch == 0 && (items >= kPersistentItemsPerSlot * resident ||
                                                  (S >= kPersistentMinStates &&
                                                   items >= kPersistentItemsPerSlotLarge * resident)));
  p.workgroups = p.persistent ? (resident < items ? resident : items) : items;
  p.lds_batch = B;
  return p;
}

template <int S, int TW, int TH, int MODE, int B>
static void launch_fwd_m(const CompositeArgs &a, int launch, int64_t items, hipStream_t st) {
  const CompositePlan p = plan_fwd_m<S, TW, TH, MODE, B>(launch, items);
  if (!p.persistent) {
    k_composite<S, TW, TH, MODE, false, B><<<(unsigned)p.workgroups, kBlock, 0, st>>>(a);
    return;
  }
  launch_zero_queues(a.queues, st);
  k_composite<S, TW, TH, MODE, true, B><<<(unsigned)p.workgroups, kBlock, 0, st>>>(a);
}

// LDS batch variants: 128, 256 and 512 entries for groups of 4 or more states
// in image and PSNR mode; 256 everywhere else (results do not depend on it).
template <int S, int MODE>
constexpr bool has_batch_variants() { return S >= 4 && (MODE == 0 || MODE == 1); }

template <typename F, int TW, int TH, int MODE, int S, typename... A>
static void run_b(int B, A &&...args) {
  if constexpr (has_batch_variants<S, MODE>()) {
    if (B == 128) { F::template run<S, TW, TH, MODE, 128>(args...); return; }
    if (B == 512) { F::template run<S, TW, TH, MODE, 512>(args...); return; }
  }
  F::template run<S, TW, TH, MODE, kBlock>(args...);
}

// Calls F::run<S, TW, TH, MODE, B>(args...) for the runtime shape; false if unsupported.
template <typename F, int TW, int TH, int MODE, typename... A>
static bool dispatch_s(int S, int B, A &&...args) {
  switch (S) {
    case 1: run_b<F, TW, TH, MODE, 1>(B, args...); return true;
    case 2: run_b<F, TW, TH, MODE, 2>(B, args...); return true;
    case 4: run_b<F, TW, TH, MODE, 4>(B, args...); return true;
    case 8: run_b<F, TW, TH, MODE, 8>(B, args...); return true;
    case 16: run_b<F, TW, TH, MODE, 16>(B, args...); return true;
    case 32: run_b<F, TW, TH, MODE, 32>(B, args...); return true;
    default: return false;
  }
}

template <typename F, int TW, int TH, typename... A>
static bool dispatch_m(int S, int B, int mode, A &&...args) {
  if (mode == 0) return dispatch_s<F, TW, TH, 0>(S, B, args...);
  if (mode == 1) return dispatch_s<F, TW, TH, 1>(S, B, args...);
  return dispatch_s<F, TW, TH, 2>(S, B, args...);
}

template <typename F, typename... A>
static bool dispatch_shape(int S, int B, int tile_w, int tile_h, int mode, A &&...args) {
  if (tile_w == 16 && tile_h == 16) return dispatch_m<F, 16, 16>(S, B, mode, args...);
  if (tile_w == 32 && tile_h == 8) return dispatch_m<F, 32, 8>(S, B, mode, args...);
  return false;
}

struct LaunchFwd {
  template <int S, int TW, int TH, int MODE, int B>
  static void run(const CompositeArgs &a, int launch, int64_t items, hipStream_t st) {
    launch_fwd_m<S, TW, TH, MODE, B>(a, launch, items, st);
  }
};

struct PlanFwd {
  template <int S, int TW, int TH, int MODE, int B>
  static void run(int launch, int64_t items, CompositePlan *out) {
    *out = plan_fwd_m<S, TW, TH, MODE, B>(launch, items);
  }
};

int launch_composite(const CompositeArgs &a, int S, int tile_w, int tile_h, int mode, int launch, int lds_batch,
                     hipStream_t st) {
  const int64_t items = work_items(a.tiles_x * a.tiles_y, a.groups);
  if (items <= 0) return 0;
  if (launch != 2 && !a.queues) return 1;
  return dispatch_shape<LaunchFwd>(S, lds_batch, tile_w, tile_h, mode, a, launch, items, st) ? 0 : 1;
}

int plan_composite(int S, int tile_w, int tile_h, int tiles, int groups, int launch, int lds_batch,
                   CompositePlan *out) {
  const int64_t items = work_items(tiles, groups);
  *out = CompositePlan{false, 0, 0, kBlock};
  if (items <= 0) return 0;
  return dispatch_shape<PlanFwd>(S, lds_batch, tile_w, tile_h, 0, launch, items, out) ? 0 : 1;
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
  const int64_t total = work_items(a.tiles_x * a.tiles_y, a.groups);
  if (total <= 0) return 0;
  const unsigned blocks = (unsigned)total;
  if (tile_w == 16 && tile_h == 16) return launch_bwd_s<16, 16>(a, S, blocks, st);
  if (tile_w == 32 && tile_h == 8) return launch_bwd_s<32, 8>(a, S, blocks, st);
  return 1;
}

}  // namespace dgs
