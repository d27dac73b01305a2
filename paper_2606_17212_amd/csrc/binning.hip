// Tile binning: per-Gaussian instance counts in depth order, instance
// emission, per-tile ranges, the per-(state group, packet, layer) delivery
// bit table, and the per-state compaction of delivered Gaussians.
//
// Gaussians are first sorted by (depth bits, index); instances are emitted in
// that order and then sorted stably by tile id alone, which yields the
// (tile, depth, index) order with a sort over 12-13 key bits instead of 44-45.
#include "common.h"
#include "kernels.h"

namespace dgs {

__global__ void k_clear_header(Header *h, unsigned long long capacity) {
  h->instances = 0ull;
  h->capacity = capacity;
  h->overflow = 0u;
  h->n_active = 0u;
}

void launch_clear_header(Header *h, unsigned long long capacity, hipStream_t st) {
  k_clear_header<<<1, 1, 0, st>>>(h, capacity);
}

__global__ void __launch_bounds__(kBlock)
k_count(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect,
        const unsigned *__restrict__ n_active, int grid_n, uint32_t *__restrict__ cnt) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= grid_n) return;
  const int nact = n_active ? (int)*n_active : grid_n;
  uint32_t c = 0;
  if (j < nact && dkey[j] != 0xFFFFFFFFu) {
    const uint2 r = rect[dval[j]];
    c = ((r.y & 0xFFFFu) - (r.x & 0xFFFFu)) * ((r.y >> 16) - (r.x >> 16));
  }
  cnt[j] = c;
}

void launch_count(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                  int grid_n, uint32_t *cnt, hipStream_t st) {
  if (grid_n <= 0) return;
  k_count<<<(unsigned)ceil_div(grid_n, kBlock), kBlock, 0, st>>>(dkey, dval, rect, n_active, grid_n, cnt);
}

// Emission: workgroup b writes the instances of the 256 depth-sorted
// Gaussians [256 b, 256 b + 256) -- one contiguous output range -- with
// consecutive lanes writing consecutive instances; each lane finds the
// Gaussian owning its output position by binary search over the workgroup's
// offsets in LDS, then its tile inside that Gaussian's rectangle (row-major).
__global__ void __launch_bounds__(kBlock)
k_emit(const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect, const uint32_t *__restrict__ off,
       const uint32_t *__restrict__ cnt, const unsigned *__restrict__ n_active, int grid_n, int tiles_x,
       Header *h, uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval) {
  __shared__ uint32_t s_off[kBlock + 1];
  __shared__ uint32_t s_id[kBlock];
  __shared__ uint32_t s_x0y0[kBlock];
  __shared__ uint32_t s_nx[kBlock];
  const int nact = n_active ? (int)*n_active : grid_n;
  const int j0 = blockIdx.x * kBlock;
  if (j0 >= nact) return;  // uniform
  const int tid = threadIdx.x;
  const int nloc = (nact - j0) < kBlock ? (nact - j0) : kBlock;
  if (tid < nloc) {
    const int j = j0 + tid;
    const uint32_t id = dval[j];
    const uint2 r = rect[id];
    s_off[tid] = off[j];
    s_id[tid] = id;
    s_x0y0[tid] = r.x;
    s_nx[tid] = (r.y & 0xFFFFu) - (r.x & 0xFFFFu);
    if (tid == nloc - 1) s_off[nloc] = off[j] + cnt[j];
  }
  __syncthreads();
  const unsigned long long begin = s_off[0], end = s_off[nloc];
  if (end > h->capacity) {  // the scan's total is checked against the same capacity
    if (tid == 0) h->overflow = 1u;
    return;
  }
  for (unsigned long long p = begin + tid; p < end; p += kBlock) {
    // last local index whose offset <= p (entries with zero count share offsets)
    int lo = 0, hi = nloc - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((unsigned long long)s_off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    const uint32_t k = (uint32_t)(p - s_off[lo]);
    const uint32_t nx = s_nx[lo];
    const uint32_t xy = s_x0y0[lo];
    const uint32_t dy = k / nx, dx = k - dy * nx;
    tkey[p] = ((xy >> 16) + dy) * (uint32_t)tiles_x + (xy & 0xFFFFu) + dx;
    tval[p] = s_id[lo];
  }
}

void launch_emit(const uint32_t *dval, const uint2 *rect, const uint32_t *off, const uint32_t *cnt,
                 const unsigned *n_active, int grid_n, int tiles_x, Header *h, uint32_t *tkey,
                 uint32_t *tval, hipStream_t st) {
  if (grid_n <= 0) return;
  k_emit<<<(unsigned)ceil_div(grid_n, kBlock), kBlock, 0, st>>>(dval, rect, off, cnt, n_active, grid_n,
                                                                tiles_x, h, tkey, tval);
}

__global__ void __launch_bounds__(kBlock) k_zero_u2(uint2 *p, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = make_uint2(0u, 0u);
}

__global__ void __launch_bounds__(kBlock)
k_ranges(const uint32_t *__restrict__ tkey, const Header *__restrict__ h, int64_t cap, int tiles,
         uint2 *__restrict__ ranges) {
  // After an overflow the instance arrays are incomplete: every range stays
  // empty, so no consumer reads an unwritten entry.
  if (h->overflow) return;
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int64_t m = (int64_t)h->instances;
  if (m > cap) m = cap;
  if (p >= m) return;
  const uint32_t t = tkey[p];
  if (t >= (uint32_t)tiles) return;
  if (p == 0 || tkey[p - 1] != t) ranges[t].x = (uint32_t)p;
  if (p == m - 1 || tkey[p + 1] != t) ranges[t].y = (uint32_t)(p + 1);
}

void launch_ranges(const uint32_t *tkey, const Header *h, int64_t cap, int tiles, uint2 *ranges,
                   hipStream_t st) {
  k_zero_u2<<<(unsigned)ceil_div(tiles, kBlock), kBlock, 0, st>>>(ranges, tiles);
  if (cap > 0) k_ranges<<<(unsigned)ceil_div(cap, kBlock), kBlock, 0, st>>>(tkey, h, cap, tiles, ranges);
}

// visbits[g][p*4 + l], bit s set iff layer l of packet p is delivered in
// state order[g*S + s] (l < code).
__global__ void __launch_bounds__(kBlock)
k_visbits(const uint8_t *__restrict__ codes, const uint32_t *__restrict__ order, int num_states, int P, int S,
          int groups, uint32_t *__restrict__ visbits) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t P4 = (int64_t)P * 4;
  if (idx >= (int64_t)groups * P4) return;
  const int g = (int)(idx / P4);
  const int pl = (int)(idx - (int64_t)g * P4);
  const int p = pl >> 2, l = pl & 3;
  uint32_t bits = 0;
  for (int s = 0; s < S; ++s) {
    const int k = g * S + s;
    if (k >= num_states) break;
    const int w = order ? (int)order[k] : k;
    if (l < (int)codes[(int64_t)w * P + p]) bits |= 1u << s;
  }
  visbits[idx] = bits;
}

void launch_visbits(const uint8_t *codes, const uint32_t *order, int num_states, int P, int S,
                    uint32_t *visbits, hipStream_t st) {
  const int groups = (int)ceil_div(num_states, S);
  const int64_t total = (int64_t)groups * P * 4;
  if (total <= 0) return;
  k_visbits<<<(unsigned)ceil_div(total, kBlock), kBlock, 0, st>>>(codes, order, num_states, P, S, groups,
                                                                  visbits);
}

// Gaussians per (packet, layer) of the binned scene.
__global__ void __launch_bounds__(kBlock)
k_plhist(const uint16_t *__restrict__ packet_layer, int n, int P4, uint32_t *__restrict__ hist) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int pl = packet_layer[i];
  if (pl < P4) atomicAdd(hist + pl, 1u);
}

__global__ void __launch_bounds__(kBlock) k_zero_u32(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

void launch_plhist(const uint16_t *packet_layer, int n, int P, uint32_t *hist, hipStream_t st) {
  const int P4 = P * 4;
  k_zero_u32<<<(unsigned)ceil_div(P4, kBlock), kBlock, 0, st>>>(hist, P4);
  if (n > 0) k_plhist<<<(unsigned)ceil_div(n, kBlock), kBlock, 0, st>>>(packet_layer, n, P4, hist);
}

// Present count of every state (one workgroup per state) from the
// (packet, layer) histogram.
__global__ void __launch_bounds__(kBlock)
k_state_counts(const uint8_t *__restrict__ codes, const uint32_t *__restrict__ hist, int P,
               uint32_t *__restrict__ cnt) {
  const int w = blockIdx.x;
  uint32_t c = 0;
  for (int p = threadIdx.x; p < P; p += kBlock) {
    const int code = codes[(int64_t)w * P + p];
    const uint4 h = reinterpret_cast<const uint4 *>(hist)[p];
    c += (code > 0 ? h.x : 0u) + (code > 1 ? h.y : 0u) + (code > 2 ? h.z : 0u) + (code > 3 ? h.w : 0u);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, kWave);
  __shared__ uint32_t part[4];
  if (__lane_id() == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[w] = part[0] + part[1] + part[2] + part[3];
}

// One workgroup: states ordered by increasing present count (ties by index),
// so that the S states of a group have similar list-walk depths.
__global__ void __launch_bounds__(1024)
k_state_rank(const uint32_t *__restrict__ cnt_g, int num_states, uint32_t *__restrict__ order) {
  extern __shared__ uint32_t cnt[];
  for (int w = threadIdx.x; w < num_states; w += blockDim.x) cnt[w] = cnt_g[w];
  __syncthreads();
  for (int w = threadIdx.x; w < num_states; w += blockDim.x) {
    const uint32_t cw = cnt[w];
    int rank = 0;
    for (int v = 0; v < num_states; ++v) {
      const uint32_t cv = cnt[v];
      rank += (cv < cw || (cv == cw && v < w)) ? 1 : 0;
    }
    order[rank] = (uint32_t)w;
  }
}

__global__ void __launch_bounds__(kBlock) k_iota(uint32_t *p, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

void launch_state_order(const uint8_t *codes, const uint32_t *hist, int num_states, int P, uint32_t *cnt,
                        uint32_t *order, hipStream_t st) {
  if (num_states <= 0) return;
  if (num_states > kMaxOrderedStates) {  // identity order beyond the LDS-resident ranking
    k_iota<<<(unsigned)ceil_div(num_states, kBlock), kBlock, 0, st>>>(order, num_states);
    return;
  }
  k_state_counts<<<num_states, kBlock, 0, st>>>(codes, hist, P, cnt);
  k_state_rank<<<1, 1024, sizeof(uint32_t) * num_states, st>>>(cnt, num_states, order);
}

// One workgroup: tiles ordered by decreasing list length, bucketed by
// floor(log2(length + 1)) (order inside a bucket is arbitrary: every work
// item writes disjoint outputs, so the processing order never changes results).
__global__ void __launch_bounds__(1024)
k_tile_order(const uint2 *__restrict__ ranges, int tiles, uint32_t *__restrict__ order) {
  __shared__ uint32_t bcount[33];
  __shared__ uint32_t bstart[33];
  if (threadIdx.x < 33) bcount[threadIdx.x] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < tiles; t += blockDim.x) {
    const uint2 r = ranges[t];
    const uint32_t len = r.y - r.x;
    const int b = 32 - __clz(len);  // 0 for empty
    atomicAdd(&bcount[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int b = 32; b >= 0; --b) {  // heaviest bucket first
      bstart[b] = acc;
      acc += bcount[b];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tiles; t += blockDim.x) {
    const uint2 r = ranges[t];
    const int b = 32 - __clz(r.y - r.x);
    order[atomicAdd(&bstart[b], 1u)] = (uint32_t)t;
  }
}

void launch_tile_order(const uint2 *ranges, int tiles, uint32_t *order, hipStream_t st) {
  if (tiles <= 0) return;
  k_tile_order<<<1, 1024, 0, st>>>(ranges, tiles, order);
}

__global__ void __launch_bounds__(kBlock)
k_present_flags(const uint8_t *__restrict__ codes_row, const uint16_t *__restrict__ packet_layer, int n,
                int P, uint32_t *__restrict__ flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint16_t pl = packet_layer[i];
  const int p = pl >> 2;
  flags[i] = (p < P && (int)(pl & 3u) < (int)codes_row[p]) ? 1u : 0u;
}

void launch_present_flags(const uint8_t *codes_row, const uint16_t *packet_layer, int n, int P,
                          uint32_t *flags, hipStream_t st) {
  if (n <= 0) return;
  k_present_flags<<<(unsigned)ceil_div(n, kBlock), kBlock, 0, st>>>(codes_row, packet_layer, n, P, flags);
}

__global__ void __launch_bounds__(kBlock)
k_present_scatter(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ off, int n,
                  uint32_t *__restrict__ list, const unsigned long long *__restrict__ total, Header *h) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i == 0) h->n_active = (unsigned)*total;
  if (i >= n) return;
  if (flags[i]) list[off[i]] = (uint32_t)i;
}

void launch_present_scatter(const uint32_t *flags, const uint32_t *off, int n, uint32_t *list,
                            const unsigned long long *total, Header *h, hipStream_t st) {
  k_present_scatter<<<(unsigned)ceil_div(n > 0 ? n : 1, kBlock), kBlock, 0, st>>>(flags, off, n, list, total, h);
}

__global__ void __launch_bounds__(kBlock) k_fill_f32(float *p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_f32(float *p, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return;
  k_fill_f32<<<(unsigned)ceil_div(n, kBlock), kBlock, 0, st>>>(p, n, v);
}

__global__ void k_fill_u64(unsigned long long *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

void launch_fill_u64(unsigned long long *p, int n, hipStream_t st) { k_fill_u64<<<1, 64, 0, st>>>(p, n); }

}  // namespace dgs
