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

__global__ void __launch_bounds__(kBlock)
k_emit(const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect, const uint32_t *__restrict__ off,
       const uint32_t *__restrict__ cnt, const unsigned *__restrict__ n_active, int grid_n, int tiles_x,
       Header *h, uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= grid_n) return;
  const int nact = n_active ? (int)*n_active : grid_n;
  if (j >= nact) return;
  const uint32_t c = cnt[j];
  if (c == 0) return;
  const unsigned long long o0 = off[j];
  if (o0 + c > h->capacity) {
    h->overflow = 1u;
    return;
  }
  const uint32_t id = dval[j];
  const uint2 r = rect[id];
  const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu, y1 = r.y >> 16;
  uint32_t o = (uint32_t)o0;
  for (uint32_t ty = y0; ty < y1; ++ty)
    for (uint32_t tx = x0; tx < x1; ++tx) {
      tkey[o] = ty * (uint32_t)tiles_x + tx;
      tval[o] = id;
      ++o;
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
// state g*S + s (l < code).
__global__ void __launch_bounds__(kBlock)
k_visbits(const uint8_t *__restrict__ codes, int num_states, int P, int S, int groups,
          uint32_t *__restrict__ visbits) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t P4 = (int64_t)P * 4;
  if (idx >= (int64_t)groups * P4) return;
  const int g = (int)(idx / P4);
  const int pl = (int)(idx - (int64_t)g * P4);
  const int p = pl >> 2, l = pl & 3;
  uint32_t bits = 0;
  for (int s = 0; s < S; ++s) {
    const int w = g * S + s;
    if (w < num_states && l < (int)codes[(int64_t)w * P + p]) bits |= 1u << s;
  }
  visbits[idx] = bits;
}

void launch_visbits(const uint8_t *codes, int num_states, int P, int S, uint32_t *visbits, hipStream_t st) {
  const int groups = (int)ceil_div(num_states, S);
  const int64_t total = (int64_t)groups * P * 4;
  if (total <= 0) return;
  k_visbits<<<(unsigned)ceil_div(total, kBlock), kBlock, 0, st>>>(codes, num_states, P, S, groups, visbits);
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
