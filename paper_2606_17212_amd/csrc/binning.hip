// Tile binning: per-Gaussian instance counts in depth order, instance
// emission, per-tile ranges, the per-(state group, packet, layer) delivery
// bit table, and the per-state compaction of delivered Gaussians.
//
// Gaussians are first sorted by (depth bits, index); instances are emitted in
// that order and then sorted stably by tile id alone, which yields the
// (tile, depth, index) order with a sort over 12-13 key bits instead of 44-45.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace dgs {

__global__ void __launch_bounds__(kBlock) k_zero_u32(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

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

// Which of the tile's four 8x8 wave blocks a Gaussian can reach with
// alpha >= 1/255: its pixel rectangle must overlap the block, and the largest
// exponent q' over the block's pixel centres must not fall below log2(1/255)
// by more than a rounding margin.  Pixels outside reached blocks would all be
// skipped by the per-pixel test, so the mask never changes a result.
__device__ inline uint32_t block_reach_mask(const float4 &r0, const float4 &r1, const uint2 &pb, uint32_t tx,
                                            uint32_t ty, int tile_w, int tile_h) {
  const int tpx = (int)tx * tile_w, tpy = (int)ty * tile_h;
  const int x0 = (int)(pb.x & 0xFFFFu) - tpx, y0 = (int)(pb.x >> 16) - tpy;
  const int x1 = (int)(pb.y & 0xFFFFu) - tpx, y1 = (int)(pb.y >> 16) - tpy;
  const float need = kQSkip - 0.01f - r0.z;
  const float ia = -0.5f * __builtin_amdgcn_rcpf(r1.x), ic = -0.5f * __builtin_amdgcn_rcpf(r1.z);
  const float ftx = (float)tpx + 0.5f, fty = (float)tpy + 0.5f;
  if (box_all_reach(r1.x, r1.y, r1.z, r0.x - (ftx + (float)(tile_w - 1)), r0.x - ftx, r0.y - (fty + (float)(tile_h - 1)),
                    r0.y - fty, need))
    return 0xFu;  // every pixel of the tile reached
  uint32_t mask = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int bx = wave_block_x0(w, tile_w), by = wave_block_y0(w, tile_w);
    if (x0 < bx + 8 && x1 > bx && y0 < by + 8 && y1 > by) {
      const float cx0 = (float)(tpx + bx) + 0.5f, cy0 = (float)(tpy + by) + 0.5f;
      if (box_reaches(r1.x, r1.y, r1.z, ia, ic, r0.x - (cx0 + 7.0f), r0.x - cx0, r0.y - (cy0 + 7.0f), r0.y - cy0,
                      need))
        mask |= 1u << w;
    }
  }
  (void)tile_h;
  return mask;
}

__device__ inline uint32_t wave_block_mask(uint32_t id, uint32_t tx, uint32_t ty, int tile_w, int tile_h,
                                           const float4 *rec0, const float4 *rec1, const uint2 *pbox) {
  return block_reach_mask(rec0[id], rec1[id], pbox[id], tx, ty, tile_w, tile_h);
}

// Emission: one wave per depth-sorted Gaussian (grid-stride); its lanes write
// the Gaussian's instances [off, off + count) -- tiles of its rectangle in
// row-major order -- to consecutive addresses, each with the tile id as key
// and the Gaussian id plus its wave-block reach mask as value.
__global__ void __launch_bounds__(kBlock)
k_emit(const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect, const uint32_t *__restrict__ off,
       const uint32_t *__restrict__ cnt, const unsigned *__restrict__ n_active, int grid_n, int tiles_x,
       int tile_w, int tile_h, const float4 *__restrict__ rec0, const float4 *__restrict__ rec1,
       const uint2 *__restrict__ pbox, Header *h, uint32_t *__restrict__ tkey, uint32_t *__restrict__ tval) {
  const int nact = n_active ? (int)*n_active : grid_n;
  const int lane = __lane_id();
  const int wave = (int)(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
  const int nwaves = (int)(gridDim.x * (kBlock / kWave));
  const unsigned long long capacity = h->capacity;
  for (int j = wave; j < nact; j += nwaves) {
    const uint32_t c = cnt[j];
    if (c == 0) continue;
    const unsigned long long o0 = off[j];
    if (o0 + c > capacity) {
      if (lane == 0) h->overflow = 1u;
      continue;
    }
    const uint32_t id = dval[j];
    const uint2 r = rect[id];
    const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16;
    const uint32_t nx = (r.y & 0xFFFFu) - x0;
    for (uint32_t k = lane; k < c; k += kWave) {
      const uint32_t dy = k / nx, dx = k - dy * nx;
      const uint32_t tx = x0 + dx, ty = y0 + dy;
      tkey[o0 + k] = ty * (uint32_t)tiles_x + tx;
      tval[o0 + k] = id | (wave_block_mask(id, tx, ty, tile_w, tile_h, rec0, rec1, pbox) << kMaskShift);
    }
  }
}

void launch_emit(const uint32_t *dval, const uint2 *rect, const uint32_t *off, const uint32_t *cnt,
                 const unsigned *n_active, int grid_n, int tiles_x, int tile_w, int tile_h, const float4 *rec0,
                 const float4 *rec1, const uint2 *pbox, Header *h, uint32_t *tkey, uint32_t *tval,
                 hipStream_t st) {
  if (grid_n <= 0) return;
  // one wave per Gaussian, up to 8192 workgroups striding over the rest
  const int64_t blocks = ceil_div(grid_n, kBlock / kWave) < 8192 ? ceil_div(grid_n, kBlock / kWave) : 8192;
  k_emit<<<(unsigned)blocks, kBlock, 0, st>>>(dval, rect, off, cnt, n_active, grid_n, tiles_x, tile_w, tile_h,
                                              rec0, rec1, pbox, h, tkey, tval);
}

// Tile coverage as a 2D difference array: +1 at (x0, y0) and (x1, y1), -1 at
// (x1, y0) and (x0, y1) of every binned Gaussian's rectangle; its 2D prefix
// sum is the instance count of each tile.  Workgroups accumulate in LDS when
// the array fits and flush non-zero entries with one global atomic each.

__global__ void __launch_bounds__(kBlock)
k_tile_diff(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect,
            const unsigned *__restrict__ n_active, int grid_n, int tiles_x, int tiles_y, uint32_t *__restrict__ diff) {
  __shared__ uint32_t sd[kDiffLds];
  const int nx = tiles_x + 1, ne = (tiles_x + 1) * (tiles_y + 1);
  const bool in_lds = ne <= kDiffLds;
  if (in_lds)
    for (int k = threadIdx.x; k < ne; k += kBlock) sd[k] = 0u;
  __syncthreads();
  const int nact = n_active ? (int)*n_active : grid_n;
  uint32_t *d = in_lds ? sd : diff;
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < nact; j += gridDim.x * kBlock) {
    if (dkey[j] == 0xFFFFFFFFu) continue;
    const uint2 r = rect[dval[j]];
    const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16;
    if (x1 <= x0 || y1 <= y0) continue;
    atomicAdd(d + y0 * nx + x0, 1u);
    atomicAdd(d + y0 * nx + x1, 0xFFFFFFFFu);
    atomicAdd(d + y1 * nx + x0, 0xFFFFFFFFu);
    atomicAdd(d + y1 * nx + x1, 1u);
  }
  if (!in_lds) return;
  __syncthreads();
  for (int k = threadIdx.x; k < ne; k += kBlock)
    if (sd[k]) atomicAdd(diff + k, sd[k]);
}

// One workgroup: 2D inclusive prefix sum of the difference array (rows, then
// columns) -> instance count per tile.
__global__ void __launch_bounds__(1024)
k_tile_prefix(uint32_t *__restrict__ diff, int tiles_x, int tiles_y, uint32_t *__restrict__ tcnt) {
  const int nx = tiles_x + 1;
  for (int y = threadIdx.x; y < tiles_y; y += blockDim.x) {
    uint32_t acc = 0;
    for (int x = 0; x < tiles_x; ++x) {
      acc += diff[y * nx + x];
      diff[y * nx + x] = acc;
    }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < tiles_x; x += blockDim.x) {
    uint32_t acc = 0;
    for (int y = 0; y < tiles_y; ++y) {
      acc += diff[y * nx + x];
      tcnt[y * tiles_x + x] = acc;
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_ranges_from_counts(const uint32_t *__restrict__ tcnt, const uint32_t *__restrict__ tstart, int tiles,
                     const Header *__restrict__ h, uint2 *__restrict__ ranges) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= tiles) return;
  // after an overflow the instance arrays are incomplete: every range is empty
  ranges[t] = h->overflow ? make_uint2(0u, 0u) : make_uint2(tstart[t], tstart[t] + tcnt[t]);
}

// One workgroup, the whole difference array in LDS: 2D prefix (rows, then
// columns) -> instances per tile, exclusive scan over tiles -> [start, end)
// per tile, all without leaving the workgroup (used when the array fits LDS).
__global__ void __launch_bounds__(1024)
k_tile_ranges_lds(const uint32_t *__restrict__ diff, int tiles_x, int tiles_y, Header *__restrict__ h,
                  uint2 *__restrict__ ranges) {
  __shared__ uint32_t sd[kDiffLds];
  __shared__ uint32_t wsum[16];
  __shared__ unsigned long long wtot[16];
  if (threadIdx.x < 16) {
    wsum[threadIdx.x] = 0u;
    wtot[threadIdx.x] = 0ull;
  }
  const int nx = tiles_x + 1, ne = (tiles_x + 1) * (tiles_y + 1), tiles = tiles_x * tiles_y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int k = tid; k < ne; k += 1024) sd[k] = diff[k];
  __syncthreads();
  for (int y = tid; y < tiles_y; y += 1024) {
    uint32_t acc = 0;
    for (int x = 0; x < tiles_x; ++x) {
      acc += sd[y * nx + x];
      sd[y * nx + x] = acc;
    }
  }
  __syncthreads();
  for (int x = tid; x < tiles_x; x += 1024) {
    uint32_t acc = 0;
    for (int y = 0; y < tiles_y; ++y) {
      acc += sd[y * nx + x];
      sd[y * nx + x] = acc;
    }
  }
  __syncthreads();
  // counts of tile t = sd[(t / tiles_x) * nx + t % tiles_x]; each thread scans
  // a contiguous run of tiles, runs are combined by wave and workgroup scans
  const int per = (tiles + 1023) / 1024;
  const int t0 = tid * per;
  uint32_t run = 0;
  unsigned long long run64 = 0;  // the total may exceed 32 bits; the ranges only matter when it does not
  for (int k = 0; k < per; ++k) {
    const int t = t0 + k;
    if (t < tiles) {
      const uint32_t c = sd[(t / tiles_x) * nx + t % tiles_x];
      run += c;
      run64 += c;
    }
  }
  const uint32_t incl = wave_incl_scan(run);
  for (int d = 32; d >= 1; d >>= 1) run64 += __shfl_xor(run64, d, kWave);
  if (lane == 63) wsum[w] = incl;
  if (lane == 0) wtot[w] = run64;
  __syncthreads();
  uint32_t off = 0;
  unsigned long long total = 0;
  for (int k = 0; k < w; ++k) off += wsum[k];
  for (int k = 0; k < 16; ++k) total += wtot[k];
  uint32_t start = off + incl - run;
  // the instance count of this binning; more than the capacity is an
  // overflow, after which every range is empty
  const bool over = total > h->capacity;
  if (tid == 0) {
    h->instances = total;
    if (over) h->overflow = 1u;
  }
  for (int k = 0; k < per; ++k) {
    const int t = t0 + k;
    if (t >= tiles) break;
    const uint32_t c = sd[(t / tiles_x) * nx + t % tiles_x];
    ranges[t] = over ? make_uint2(0u, 0u) : make_uint2(start, start + c);
    start += c;
  }
}

bool tile_ranges_in_lds(int tiles_x, int tiles_y) {
  return (int64_t)(tiles_x + 1) * (tiles_y + 1) <= kDiffLds && (int64_t)tiles_x * tiles_y <= kChunkTiles;
}

// ---------------------------------------------------------------------------
// One-pass stable scatter of the tile instances (used when the tile grid fits
// LDS).  The depth-sorted Gaussians are cut into chunks of kChunk; one wave
// per chunk counts the chunk's instances per tile, the counts are turned into
// each chunk's first slot in every tile's range (ranges[t].x plus the counts
// of the earlier chunks), and one wave per chunk then walks its Gaussians in
// depth order writing every instance to its tile's next slot.  Within a tile
// the instances end up in depth order (chunk by chunk, then in order inside
// the chunk): the order a stable sort by tile of the depth-ordered emission
// gives.  The tiles of one Gaussian are distinct, so the per-tile slot
// counters in LDS need no atomics; successive Gaussians are ordered by the
// wave's program order.

// The 64 Gaussians [jb, jb + 64) of a wave, one per lane: id and tile
// rectangle (zero for culled or missing ones), and the records the reach
// masks need.
struct WaveGaussians {
  uint32_t id, rx, ry;
  float4 r0, r1;
  uint2 pb;
};

template <bool RECORDS>
__device__ __forceinline__ WaveGaussians load_wave_gaussians(const uint32_t *__restrict__ dkey,
                                                             const uint32_t *__restrict__ dval,
                                                             const uint2 *__restrict__ rect, int j, int j1,
                                                             const float4 *__restrict__ rec0,
                                                             const float4 *__restrict__ rec1,
                                                             const uint2 *__restrict__ pbox) {
  WaveGaussians q{};
  if (j < j1 && dkey[j] != 0xFFFFFFFFu) {
    q.id = dval[j];
    const uint2 r = rect[q.id];
    q.rx = r.x;
    q.ry = r.y;
    if (RECORDS) {
      q.r0 = rec0[q.id];
      q.r1 = rec1[q.id];
      q.pb = pbox[q.id];
    }
  }
  return q;
}

// Visits the tiles of the wave's Gaussians g = 0..ng-1 in order, lanes over
// each rectangle (row-major); f(g, tile, tx, ty) runs once per instance.
template <typename F>
__device__ __forceinline__ void for_wave_instances(const WaveGaussians &q, int ng, int tiles_x, F &&f) {
  for (int g = 0; g < ng; ++g) {
    const uint32_t gx = __builtin_amdgcn_readlane(q.rx, g), gy = __builtin_amdgcn_readlane(q.ry, g);
    const uint32_t x0 = gx & 0xFFFFu, y0 = gx >> 16, x1 = gy & 0xFFFFu, y1 = gy >> 16;
    if (x1 <= x0 || y1 <= y0) continue;  // culled (all zero) or empty
    const uint32_t nx = x1 - x0, area = nx * (y1 - y0);
    for (uint32_t k = __lane_id(); k < area; k += kWave) {
      const uint32_t dy = k / nx, tx = x0 + (k - dy * nx), ty = y0 + dy;
      f(g, ty * (uint32_t)tiles_x + tx, tx, ty);
    }
  }
}

__device__ __forceinline__ uint32_t readlane_u(uint32_t v, int g) { return __builtin_amdgcn_readlane(v, g); }
__device__ __forceinline__ float readlane_f(float v, int g) {
  return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), g));
}

// Instances per tile of chunk c (kChunk depth-ordered Gaussians, four waves
// of kWaveGauss), counted with LDS atomics.
__global__ void __launch_bounds__(kBlock)
k_chunk_hist(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect,
             const unsigned *__restrict__ n_active, int grid_n, int tiles_x, int tiles, uint32_t *__restrict__ chist) {
  extern __shared__ uint32_t cnt[];
  const int nact = n_active ? (int)*n_active : grid_n;
  for (int t = threadIdx.x; t < tiles; t += kBlock) cnt[t] = 0u;
  __syncthreads();
  const int jb = blockIdx.x * kChunk + (threadIdx.x >> 6) * kWaveGauss;
  const int j1 = (jb + kWaveGauss) < nact ? (jb + kWaveGauss) : nact;
  if (jb < j1) {
    const WaveGaussians q = load_wave_gaussians<false>(dkey, dval, rect, jb + __lane_id(), j1, nullptr, nullptr,
                                                       nullptr);
    const int ng = j1 - jb;
    for_wave_instances(q, ng, tiles_x, [&](int, uint32_t t, uint32_t, uint32_t) { atomicAdd(&cnt[t], 1u); });
  }
  __syncthreads();
  uint32_t *row = chist + (int64_t)blockIdx.x * tiles;
  for (int t = threadIdx.x; t < tiles; t += kBlock) row[t] = cnt[t];
}

// Totals of segments of kSegChunks chunks per tile (thread = tile, y = segment).
__global__ void __launch_bounds__(kBlock)
k_chunk_segsum(const uint32_t *__restrict__ chist, int chunks, int tiles, uint32_t *__restrict__ segsum) {
  const int t = blockIdx.x * kBlock + threadIdx.x, sg = blockIdx.y;
  if (t >= tiles) return;
  const int c0 = sg * kSegChunks, c1 = (c0 + kSegChunks) < chunks ? (c0 + kSegChunks) : chunks;
  uint32_t s = 0;
  for (int c = c0; c < c1; ++c) s += chist[(int64_t)c * tiles + t];
  segsum[(int64_t)sg * tiles + t] = s;
}

// segsum[s][t] <- instances of tile t in segments before s (exclusive
// prefix over segments).  A workgroup takes 16 tiles; 16 threads per tile
// split the segments into 16 parts (reads coalesced across the 16 tiles):
// part totals, their prefix in LDS, then each part rewritten in order.
constexpr int kScanTiles = 16, kScanParts = kBlock / kScanTiles;
__global__ void __launch_bounds__(kBlock)
k_chunk_segscan(uint32_t *__restrict__ segsum, int nseg, int tiles) {
  __shared__ uint32_t part[kScanParts][kScanTiles + 1];
  const int tl = threadIdx.x % kScanTiles, pp = threadIdx.x / kScanTiles;
  const int t = blockIdx.x * kScanTiles + tl;
  const int per = (nseg + kScanParts - 1) / kScanParts;
  const int k0 = pp * per, k1 = (k0 + per) < nseg ? (k0 + per) : nseg;
  uint32_t sum = 0;
  if (t < tiles)
    for (int k = k0; k < k1; ++k) sum += segsum[(int64_t)k * tiles + t];
  part[pp][tl] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (int q = 0; q < pp; ++q) run += part[q][tl];
  if (t < tiles)
    for (int k = k0; k < k1; ++k) {
      const uint32_t v = segsum[(int64_t)k * tiles + t];
      segsum[(int64_t)k * tiles + t] = run;
      run += v;
    }
}

// chist[c][t] <- ranges[t].x + instances of tile t in chunks before c.
__global__ void __launch_bounds__(kBlock)
k_chunk_offsets(uint32_t *__restrict__ chist, const uint32_t *__restrict__ segsum, const uint2 *__restrict__ ranges,
                int chunks, int tiles) {
  const int t = blockIdx.x * kBlock + threadIdx.x, sg = blockIdx.y;
  if (t >= tiles) return;
  uint32_t base = ranges[t].x + segsum[(int64_t)sg * tiles + t];
  const int c0 = sg * kSegChunks, c1 = (c0 + kSegChunks) < chunks ? (c0 + kSegChunks) : chunks;
  for (int c = c0; c < c1; ++c) {
    const uint32_t v = chist[(int64_t)c * tiles + t];
    chist[(int64_t)c * tiles + t] = base;
    base += v;
  }
}

// Scatter of chunk c: wave w owns Gaussians [c kChunk + w kWaveGauss, +kWaveGauss).  Its
// instances of tile t go after the chunk's first slot choff[c][t] and the
// instances of tile t owned by waves < w.  The four waves' next slots per tile
// live in LDS as 16-bit counts relative to choff[c][t] (at most kWaveGauss per
// wave and tile, so the prefix over the waves fits), which is read per
// instance: half the LDS of absolute 32-bit slots, so twice the resident
// workgroups (measured faster at 2,500 tiles as well as at 8,160).
__global__ void __launch_bounds__(kBlock)
k_chunk_scatter(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect,
                const unsigned *__restrict__ n_active, int grid_n, int tiles_x, int tiles, int tile_w, int tile_h,
                const float4 *__restrict__ rec0, const float4 *__restrict__ rec1, const uint2 *__restrict__ pbox,
                const uint32_t *__restrict__ choff, const Header *__restrict__ h, uint32_t *__restrict__ tval) {
  using Slot = uint16_t;
  extern __shared__ uint32_t lds_raw[];
  Slot *rel = reinterpret_cast<Slot *>(lds_raw);  // [4][tiles]
  if (h->overflow) return;  // the ranges are empty; nothing may be written past the capacity
  const int nact = n_active ? (int)*n_active : grid_n;
  const int w = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < 4 * tiles; t += kBlock) rel[t] = 0;
  __syncthreads();
  const int jb = blockIdx.x * kChunk + w * kWaveGauss;
  const int j1 = (jb + kWaveGauss) < nact ? (jb + kWaveGauss) : nact;
  const int ng = jb < j1 ? j1 - jb : 0;
  const WaveGaussians q = load_wave_gaussians<true>(dkey, dval, rect, jb + __lane_id(), j1, rec0, rec1, pbox);
  Slot *mine = rel + w * tiles;
  // per-wave counts (each Gaussian's tiles are distinct; Gaussians in program order)
  for_wave_instances(q, ng, tiles_x, [&](int, uint32_t t, uint32_t, uint32_t) { mine[t] = (Slot)(mine[t] + 1); });
  __syncthreads();
  const uint32_t *row = choff + (int64_t)blockIdx.x * tiles;
  for (int t = threadIdx.x; t < tiles; t += kBlock) {  // counts -> first slot of each wave
    const uint32_t a = rel[t], b = rel[tiles + t], c = rel[2 * tiles + t];
    rel[t] = 0;
    rel[tiles + t] = (Slot)a;
    rel[2 * tiles + t] = (Slot)(a + b);
    rel[3 * tiles + t] = (Slot)(a + b + c);
  }
  __syncthreads();
  // per Gaussian of the wave: the reciprocals of the reach test, once
  const float ia = -0.5f * __builtin_amdgcn_rcpf(q.r1.x), ic = -0.5f * __builtin_amdgcn_rcpf(q.r1.z);
  for (int g = 0; g < ng; ++g) {
    const uint32_t gx = readlane_u(q.rx, g), gy = readlane_u(q.ry, g);
    const uint32_t x0 = gx & 0xFFFFu, y0 = gx >> 16, x1 = gy & 0xFFFFu, y1 = gy >> 16;
    if (x1 <= x0 || y1 <= y0) continue;
    const uint32_t nx = x1 - x0, area = nx * (y1 - y0);
    const uint32_t id = readlane_u(q.id, g);
    const float u = readlane_f(q.r0.x, g), v = readlane_f(q.r0.y, g), lo = readlane_f(q.r0.z, g);
    const float A = readlane_f(q.r1.x, g), B = readlane_f(q.r1.y, g), C = readlane_f(q.r1.z, g);
    const float gia = readlane_f(ia, g), gic = readlane_f(ic, g);
    const uint32_t pbx = readlane_u(q.pb.x, g), pby = readlane_u(q.pb.y, g);
    const float need = kQSkip - 0.01f - lo;
    for (uint32_t k = __lane_id(); k < area; k += kWave) {
      const uint32_t dy = k / nx, tx = x0 + (k - dy * nx), ty = y0 + dy;
      const uint32_t t = ty * (uint32_t)tiles_x + tx;
      const uint32_t slot = row[t] + (uint32_t)mine[t];
      mine[t] = (Slot)(mine[t] + 1);
      // which of the tile's four 8x8 wave blocks the Gaussian reaches (as block_reach_mask)
      const int tpx = (int)tx * tile_w, tpy = (int)ty * tile_h;
      const int px0 = (int)(pbx & 0xFFFFu) - tpx, py0 = (int)(pbx >> 16) - tpy;
      const int px1 = (int)(pby & 0xFFFFu) - tpx, py1 = (int)(pby >> 16) - tpy;
      // every pixel of the tile reached: all four blocks, no per-block search
      const float ftx = (float)tpx + 0.5f, fty = (float)tpy + 0.5f;
      const bool whole = box_all_reach(A, B, C, u - (ftx + (float)(tile_w - 1)), u - ftx,
                                       v - (fty + (float)(tile_h - 1)), v - fty, need);
      uint32_t mask = whole ? 0xFu : 0u;
#pragma unroll
      for (int wb = 0; wb < 4; ++wb) {
        if (whole) break;
        const int bx = wave_block_x0(wb, tile_w), by = wave_block_y0(wb, tile_w);
        if (px0 < bx + 8 && px1 > bx && py0 < by + 8 && py1 > by) {
          const float cx0 = (float)(tpx + bx) + 0.5f, cy0 = (float)(tpy + by) + 0.5f;
          if (box_reaches(A, B, C, gia, gic, u - (cx0 + 7.0f), u - cx0, v - (cy0 + 7.0f), v - cy0, need))
            mask |= 1u << wb;
        }
      }
      tval[slot] = id | (mask << kMaskShift);
    }
  }
}

void launch_chunk_scatter(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                          int grid_n, int tiles_x, int tiles_y, int tile_w, int tile_h, const float4 *rec0,
                          const float4 *rec1, const uint2 *pbox, const uint2 *ranges, const Header *h,
                          uint32_t *chist, uint32_t *segsum, uint32_t *tval, hipStream_t st) {
  const int chunks = (int)ceil_div(grid_n, kChunk);
  if (chunks <= 0) return;
  const int tiles = tiles_x * tiles_y;
  const int nseg = (int)ceil_div(chunks, kSegChunks);
  const dim3 tg((unsigned)ceil_div(tiles, kBlock), (unsigned)nseg);
  k_chunk_hist<<<chunks, kBlock, sizeof(uint32_t) * (size_t)tiles, st>>>(dkey, dval, rect, n_active, grid_n,
                                                                       tiles_x, tiles, chist);
  k_chunk_segsum<<<tg, kBlock, 0, st>>>(chist, chunks, tiles, segsum);
  k_chunk_segscan<<<(unsigned)ceil_div(tiles, kScanTiles), kBlock, 0, st>>>(segsum, nseg, tiles);
  k_chunk_offsets<<<tg, kBlock, 0, st>>>(chist, segsum, ranges, chunks, tiles);
  k_chunk_scatter<<<chunks, kBlock, sizeof(uint16_t) * 4 * (size_t)tiles, st>>>(
      dkey, dval, rect, n_active, grid_n, tiles_x, tiles, tile_w, tile_h, rec0, rec1, pbox, chist, h, tval);

}

void launch_tile_ranges(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                        int grid_n, int tiles_x, int tiles_y, Header *h, uint32_t *tdiff, uint32_t *tcnt,
                        uint32_t *tstart, unsigned long long *parts, uint2 *ranges, hipStream_t st) {
  const int tiles = tiles_x * tiles_y;
  const int64_t ne = (int64_t)(tiles_x + 1) * (tiles_y + 1);
  k_zero_u32<<<(unsigned)ceil_div(ne, kBlock), kBlock, 0, st>>>(tdiff, ne);
  if (grid_n > 0) {
    // enough workgroups to cover the machine, few enough to keep the LDS flushes cheap
    const int64_t per = ne <= kDiffLds ? (grid_n / 512 > 1024 ? grid_n / 512 : 1024) : 1024;
    const int blocks = (int)ceil_div(grid_n, per);
    k_tile_diff<<<blocks, kBlock, 0, st>>>(dkey, dval, rect, n_active, grid_n, tiles_x, tiles_y, tdiff);
  }
  if (ne <= kDiffLds) {
    k_tile_ranges_lds<<<1, 1024, 0, st>>>(tdiff, tiles_x, tiles_y, h, ranges);
    return;
  }
  k_tile_prefix<<<1, 1024, 0, st>>>(tdiff, tiles_x, tiles_y, tcnt);
  launch_scan_u32(tcnt, tstart, tiles, parts, nullptr, st);
  k_ranges_from_counts<<<(unsigned)ceil_div(tiles, kBlock), kBlock, 0, st>>>(tcnt, tstart, tiles, h, ranges);
}

// visbits[g][p*4 + l], bit s set iff layer l of packet p is delivered in
// state order[g*S + s] (l < code).  exact: records of a scene with
// refinement levels, where l is the delivered depth a record was projected
// at; the bit is set iff the state delivers exactly that depth (codes above
// 4 act as 4).
__global__ void __launch_bounds__(kBlock)
k_visbits(const uint8_t *__restrict__ codes, const uint32_t *__restrict__ order, int num_states, int P, int S,
          int groups, int exact, uint32_t *__restrict__ visbits) {
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
    const int code = codes[(int64_t)w * P + p];
    if (exact ? (code < 4 ? code : 4) == l + 1 : l < code) bits |= 1u << s;
  }
  visbits[idx] = bits;
}

void launch_visbits(const uint8_t *codes, const uint32_t *order, int num_states, int P, int S, bool exact,
                    uint32_t *visbits, hipStream_t st) {
  const int groups = (int)ceil_div(num_states, S);
  const int64_t total = (int64_t)groups * P * 4;
  if (total <= 0) return;
  k_visbits<<<(unsigned)ceil_div(total, kBlock), kBlock, 0, st>>>(codes, order, num_states, P, S, groups,
                                                                  exact ? 1 : 0, visbits);
}

// Gaussians per (packet, layer) of the binned scene.
__global__ void __launch_bounds__(kBlock)
k_plhist(const uint16_t *__restrict__ packet_layer, int n, int P4, uint32_t *__restrict__ hist) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int pl = packet_layer[i];
  if (pl < P4) atomicAdd(hist + pl, 1u);
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

// The list holds record ids: the Gaussian i, or with refinement levels its
// record 4 i + d at the delivered depth d (codes above 4 act as 4).
__global__ void __launch_bounds__(kBlock)
k_present_scatter(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ off, int n,
                  const uint8_t *__restrict__ codes_row, const uint16_t *__restrict__ packet_layer, int refined,
                  uint32_t *__restrict__ list, const unsigned long long *__restrict__ total, Header *h) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i == 0) h->n_active = (unsigned)*total;
  if (i >= n) return;
  if (!flags[i]) return;
  uint32_t v = (uint32_t)i;
  if (refined) {
    const int c = codes_row[packet_layer[i] >> 2];  // present: the packet is in range and c > layer
    v = 4u * (uint32_t)i + (uint32_t)((c < 4 ? c : 4) - 1);
  }
  list[off[i]] = v;
}

void launch_present_scatter(const uint32_t *flags, const uint32_t *off, int n, const uint8_t *codes_row,
                            const uint16_t *packet_layer, bool refined, uint32_t *list,
                            const unsigned long long *total, Header *h, hipStream_t st) {
  k_present_scatter<<<(unsigned)ceil_div(n > 0 ? n : 1, kBlock), kBlock, 0, st>>>(
      flags, off, n, codes_row, packet_layer, refined ? 1 : 0, list, total, h);
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

__global__ void k_zero_queues(unsigned int *q) {
  if (threadIdx.x < 8) q[threadIdx.x] = 0u;
}

void launch_zero_queues(unsigned int *queues, hipStream_t st) { k_zero_queues<<<1, 64, 0, st>>>(queues); }

}  // namespace dgs
