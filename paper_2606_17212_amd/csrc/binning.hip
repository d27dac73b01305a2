// Tile binning: per-tile ranges from the Gaussians' tile rectangles, the
// instances of the depth-sorted Gaussians put in (tile, depth, index) order,
// the per-(state group, packet, layer) delivery bit table, and the per-state
// compaction of delivered Gaussians.
//
// Gaussians are first sorted by (depth bits, index).  For tile grids of at
// most kMaxSupers super-tiles the instances are then placed by a two-level
// stable scatter (super-tile lists, then tiles); larger grids emit the
// instances in depth order and sort them stably by tile id alone, a sort over
// the tile bits instead of tile and depth bits.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace dgs {

__global__ void __launch_bounds__(kBlock) k_zero_u32(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Header reset, and up to two u32 arrays zeroed in the same launch.
__global__ void __launch_bounds__(kBlock)
k_clear_header(Header *h, unsigned long long capacity, uint32_t *za, int64_t na, uint32_t *zb, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i == 0) {
    h->instances = 0ull;
    h->capacity = capacity;
    h->overflow = 0u;
    h->n_active = 0u;
  }
  if (i < na) za[i] = 0u;
  if (i < nb) zb[i] = 0u;
}

void launch_clear_header(Header *h, unsigned long long capacity, hipStream_t st, uint32_t *za, int64_t na,
                         uint32_t *zb, int64_t nb) {
  const int64_t m = na > nb ? na : nb;
  k_clear_header<<<(unsigned)ceil_div(m > 0 ? m : 1, kBlock), kBlock, 0, st>>>(h, capacity, za, za ? na : 0, zb,
                                                                                 zb ? nb : 0);
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
__device__ inline uint32_t block_reach_mask_pre(const float4 &r0, const float4 &r1, const uint2 &pb, float need,
                                                float ia, float ic, uint32_t tx, uint32_t ty, int tile_w, int tile_h) {
  const int tpx = (int)tx * tile_w, tpy = (int)ty * tile_h;
  const int x0 = (int)(pb.x & 0xFFFFu) - tpx, y0 = (int)(pb.x >> 16) - tpy;
  const int x1 = (int)(pb.y & 0xFFFFu) - tpx, y1 = (int)(pb.y >> 16) - tpy;
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
  return mask;
}

// (need = log2(1/255) - 0.01 - log2 o; ia = -1/(2 A'), ic = -1/(2 C') of the record)
__device__ inline uint32_t block_reach_mask(const float4 &r0, const float4 &r1, const uint2 &pb, uint32_t tx,
                                            uint32_t ty, int tile_w, int tile_h) {
  const float need = kQSkip - 0.01f - r0.z;
  const float ia = -0.5f * __builtin_amdgcn_rcpf(r1.x), ic = -0.5f * __builtin_amdgcn_rcpf(r1.z);
  return block_reach_mask_pre(r0, r1, pb, need, ia, ic, tx, ty, tile_w, tile_h);
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
// the array fits and flush non-zero entries with one global atomic each.  The
// LDS array is sized at launch to the tile grid (4 (tiles_x + 1) (tiles_y + 1)
// bytes, 10.4 KB at 50 x 50 tiles), so that a workgroup fits in the LDS one
// compositing workgroup leaves when the kernel runs beside a compositing grid
// on another stream.

__global__ void __launch_bounds__(kBlock)
k_tile_diff(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect,
            const unsigned *__restrict__ n_active, int grid_n, int tiles_x, int tiles_y, uint32_t *__restrict__ diff) {
  extern __shared__ uint32_t sd[];  // (tiles_x + 1) (tiles_y + 1) entries when they fit kDiffLds, else unused
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

// h->instances holds the total of the counts; more than the capacity is an
// overflow, after which the instance arrays are incomplete and every range
// is empty.
__global__ void __launch_bounds__(kBlock)
k_ranges_from_counts(const uint32_t *__restrict__ tcnt, const uint32_t *__restrict__ tstart, int tiles,
                     Header *__restrict__ h, uint2 *__restrict__ ranges) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const bool over = h->overflow || h->instances > h->capacity;
  if (t == 0 && over) h->overflow = 1u;
  if (t >= tiles) return;
  ranges[t] = over ? make_uint2(0u, 0u) : make_uint2(tstart[t], tstart[t] + tcnt[t]);
}

// One workgroup, the whole difference array in LDS: 2D prefix (rows, then
// columns) -> instances per tile, exclusive scan over tiles -> [start, end)
// per tile, all without leaving the workgroup (used when the array fits LDS).
// A workgroup of kBlock threads with the array sized at launch: it takes the
// place of one compositing workgroup when it runs beside a compositing grid.
__global__ void __launch_bounds__(kBlock)
k_tile_ranges_lds(const uint32_t *__restrict__ diff, int tiles_x, int tiles_y, Header *__restrict__ h,
                  uint2 *__restrict__ ranges, uint32_t *__restrict__ tile_order) {
  constexpr int kWaves = kBlock / kWave;
  extern __shared__ uint32_t sd[];  // (tiles_x + 1) (tiles_y + 1) entries
  __shared__ uint32_t wsum[kWaves];
  __shared__ unsigned long long wtot[kWaves];
  __shared__ uint32_t bcount[33], bstart[33];
  if (threadIdx.x < kWaves) {
    wsum[threadIdx.x] = 0u;
    wtot[threadIdx.x] = 0ull;
  }
  const int nx = tiles_x + 1, ne = (tiles_x + 1) * (tiles_y + 1), tiles = tiles_x * tiles_y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int e = tid;
  for (; e + 3 * kBlock < ne; e += 4 * kBlock) {  // four reads in flight per thread
    const uint32_t v0 = diff[e], v1 = diff[e + kBlock], v2 = diff[e + 2 * kBlock], v3 = diff[e + 3 * kBlock];
    sd[e] = v0;
    sd[e + kBlock] = v1;
    sd[e + 2 * kBlock] = v2;
    sd[e + 3 * kBlock] = v3;
  }
  for (; e < ne; e += kBlock) sd[e] = diff[e];
  __syncthreads();
  for (int y = tid; y < tiles_y; y += kBlock) {
    uint32_t acc = 0;
    for (int x = 0; x < tiles_x; ++x) {
      acc += sd[y * nx + x];
      sd[y * nx + x] = acc;
    }
  }
  __syncthreads();
  for (int x = tid; x < tiles_x; x += kBlock) {
    uint32_t acc = 0;
    for (int y = 0; y < tiles_y; ++y) {
      acc += sd[y * nx + x];
      sd[y * nx + x] = acc;
    }
  }
  __syncthreads();
  // counts of tile t = sd[(t / tiles_x) * nx + t % tiles_x]; each thread scans
  // a contiguous run of tiles, runs are combined by wave and workgroup scans
  const int per = (tiles + kBlock - 1) / kBlock;
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
  for (int k = 0; k < kWaves; ++k) total += wtot[k];
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
  if (!tile_order) return;
  // tiles by decreasing list length, as k_tile_order (from the counts in LDS)
  if (tid < 33) bcount[tid] = 0u;
  __syncthreads();
  for (int t = tid; t < tiles; t += kBlock) {
    const uint32_t len = over ? 0u : sd[(t / tiles_x) * nx + t % tiles_x];
    atomicAdd(&bcount[32 - __clz(len)], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int q = 32; q >= 0; --q) {  // heaviest bucket first
      bstart[q] = acc;
      acc += bcount[q];
    }
  }
  __syncthreads();
  for (int t = tid; t < tiles; t += kBlock) {
    const uint32_t len = over ? 0u : sd[(t / tiles_x) * nx + t % tiles_x];
    tile_order[atomicAdd(&bstart[32 - __clz(len)], 1u)] = (uint32_t)t;
  }
}

bool tile_ranges_in_lds(int tiles_x, int tiles_y) { return (int64_t)(tiles_x + 1) * (tiles_y + 1) <= kDiffLds; }

// ---------------------------------------------------------------------------
// Two-level stable scatter of the tile instances (tile grids of at most
// kMaxSupers super-tiles of kSuper x kSuper tiles).
//
// Level 1 puts every depth-sorted Gaussian into the list of each super-tile
// its tile rectangle touches, in depth order.  Level 2 walks each super-tile's
// list in segments of kSegWave entries, one wave per segment, and writes the
// instances of the super-tile's 64 tiles: per tile, one ballot over the
// wave's 64 entries ranks the lanes that cover it, and they write
// consecutive slots of that tile's range with one store.  A tile's run of
// slots per segment is kSegWave x (the share of the super-tile a Gaussian
// covers) entries long, where scattering chunks of depth-ordered Gaussians
// straight to tiles leaves runs of a few entries per tile and partial
// cache-line writes.  Within a tile the instances end up in depth order: the
// super-tile lists keep depth order, and segments, rounds of 64 entries and
// lanes follow it.  Every kernel returns at once after an overflow (the
// ranges are empty then and the lists would not fit).

// Super-tile rectangle [sx0, sx1) x [sy0, sy1) of depth-sorted Gaussian j
// (empty past the active count or when culled).
__device__ inline void super_rect(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval,
                                  const uint2 *__restrict__ rect, int j, int nact, uint32_t &id, uint32_t &sx0,
                                  uint32_t &sy0, uint32_t &nx, uint32_t &area) {
  id = 0u;
  sx0 = sy0 = nx = area = 0u;
  if (j >= nact || dkey[j] == 0xFFFFFFFFu) return;
  id = dval[j];
  const uint2 r = rect[id];
  const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu, y1 = r.y >> 16;
  if (x1 <= x0 || y1 <= y0) return;
  sx0 = x0 / kSuper;
  sy0 = y0 / kSuper;
  nx = (x1 - 1) / kSuper + 1 - sx0;
  area = nx * ((y1 - 1) / kSuper + 1 - sy0);
}

__device__ inline uint32_t super_at(uint32_t k, uint32_t sx0, uint32_t sy0, uint32_t nx, int supers_x) {
  const uint32_t dy = k / nx;
  return (sy0 + dy) * (uint32_t)supers_x + sx0 + (k - dy * nx);
}

// Per-wave super-tile counts of one round of 64 Gaussians: every lane sets
// its bit in the wave's word of each super-tile it covers; the lowest
// covering lane then adds the word's population to cnt and clears the word.
// (A lane that finds the word already cleared by the lowest one adds zero.)
// LDS operations of one wave complete in order, so each phase sees the last.
__device__ inline void super_round_count(unsigned long long *bits, uint32_t *cnt, uint32_t sx0, uint32_t sy0,
                                         uint32_t nx, uint32_t area, int supers_x) {
  const unsigned long long me = 1ull << __lane_id(), below = lanemask_lt();
  for (uint32_t k = 0; k < area; ++k) atomicOr(&bits[super_at(k, sx0, sy0, nx, supers_x)], me);
  __builtin_amdgcn_wave_barrier();
  for (uint32_t k = 0; k < area; ++k) {
    const uint32_t s = super_at(k, sx0, sy0, nx, supers_x);
    const unsigned long long b = bits[s];
    if ((b & below) == 0ull) {
      cnt[s] += (uint32_t)__popcll(b);
      bits[s] = 0ull;
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// Level 1 counts: instances per (super-tile, chunk of kLevel1Chunk Gaussians);
// each wave takes kLevel1Chunk / 256 rounds of 64 consecutive Gaussians.
__global__ void __launch_bounds__(kBlock)
k_super_count(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect,
              const unsigned *__restrict__ n_active, int grid_n, int supers_x, int nsup, int chunks,
              const Header *__restrict__ h, uint32_t *__restrict__ scnt) {
  extern __shared__ unsigned long long lds_bits[];  // [4][nsup] words, then [4][nsup] counts
  if (h->overflow) return;
  const int w = threadIdx.x >> 6;
  unsigned long long *bits = lds_bits + w * nsup;
  uint32_t *cnt_all = reinterpret_cast<uint32_t *>(lds_bits + 4 * nsup), *cnt = cnt_all + w * nsup;
  for (int s = __lane_id(); s < nsup; s += kWave) {
    bits[s] = 0ull;
    cnt[s] = 0u;
  }
  __builtin_amdgcn_wave_barrier();
  const int nact = n_active ? (int)*n_active : grid_n;
  const int jw = blockIdx.x * kLevel1Chunk + w * (kLevel1Chunk / 4);
  for (int r = 0; r < kLevel1Chunk / 4 / kWave; ++r) {
    uint32_t id, sx0, sy0, nx, area;
    super_rect(dkey, dval, rect, jw + r * kWave + __lane_id(), nact, id, sx0, sy0, nx, area);
    super_round_count(bits, cnt, sx0, sy0, nx, area, supers_x);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nsup; s += kBlock)
    scnt[(int64_t)s * chunks + blockIdx.x] =
        cnt_all[s] + cnt_all[nsup + s] + cnt_all[2 * nsup + s] + cnt_all[3 * nsup + s];
}

// Level 1: exclusive prefix over chunks of one super-tile's counts (in place)
// and its list length.  One workgroup per super-tile, a contiguous run of
// chunks per thread.
__global__ void __launch_bounds__(kBlock)
k_super_scan(uint32_t *__restrict__ scnt, int chunks, const Header *__restrict__ h, uint32_t *__restrict__ slen) {
  __shared__ uint32_t wsum[4];
  if (h->overflow) return;
  uint32_t *row = scnt + (int64_t)blockIdx.x * chunks;
  const int per = (chunks + kBlock - 1) / kBlock;
  const int c0 = threadIdx.x * per < chunks ? threadIdx.x * per : chunks;
  const int c1 = c0 + per < chunks ? c0 + per : chunks;
  uint32_t sum = 0;
  for (int c = c0; c < c1; ++c) sum += row[c];
  const uint32_t incl = wave_incl_scan(sum);
  const int w = threadIdx.x >> 6;
  if (__lane_id() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int k = 0; k < w; ++k) run += wsum[k];
  for (int c = c0; c < c1; ++c) {
    const uint32_t v = row[c];
    row[c] = run;
    run += v;
  }
  if (threadIdx.x == kBlock - 1) slen[blockIdx.x] = run;
}

// Super-tile tables from the list lengths (one workgroup, in LDS): list start
// and first level-2 segment of each super-tile, seg[nsup] = segments in all.
__device__ inline void super_tables(const uint32_t *__restrict__ slen, int nsup, uint32_t *sstart, uint32_t *seg) {
  __shared__ uint32_t wl[4], wg[4];
  // each thread owns kMaxSupers / kBlock consecutive super-tiles
  constexpr int per = kMaxSupers / kBlock;
  const int s0 = threadIdx.x * per;
  uint32_t len[per], tl = 0, tg = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    len[k] = s0 + k < nsup ? slen[s0 + k] : 0u;
    tl += len[k];
    tg += (len[k] + kSegWave - 1) / kSegWave;
  }
  const uint32_t il = wave_incl_scan(tl), ig = wave_incl_scan(tg);
  const int w = threadIdx.x >> 6;
  if (__lane_id() == kWave - 1) {
    wl[w] = il;
    wg[w] = ig;
  }
  __syncthreads();
  uint32_t rl = il - tl, rg = ig - tg;
  for (int k = 0; k < w; ++k) {
    rl += wl[k];
    rg += wg[k];
  }
#pragma unroll
  for (int k = 0; k < per; ++k) {
    if (s0 + k <= nsup) {
      sstart[s0 + k] = rl;
      seg[s0 + k] = rg;
    }
    rl += len[k];
    rg += (len[k] + kSegWave - 1) / kSegWave;
  }
  if (threadIdx.x == 0 && nsup == kMaxSupers) {  // the one entry past the last thread's run
    sstart[kMaxSupers] = wl[0] + wl[1] + wl[2] + wl[3];
    seg[kMaxSupers] = wg[0] + wg[1] + wg[2] + wg[3];
  }
  __syncthreads();
}

// Level 1 scatter: the same rounds as k_super_count; each wave's first slot
// per super-tile is the super-tile's list start + the chunk's prefix + the
// counts of the workgroup's earlier waves, and a covering lane's slot adds
// the number of lower lanes covering the same super-tile in its round.
// Workgroup 0 also writes the super-tile tables for level 2:
// tab[0..] list lengths (already there), tab[K+1..] starts, tab[2K+2..]
// first segments (K = kMaxSupers).
__global__ void __launch_bounds__(kBlock)
k_super_scatter(const uint32_t *__restrict__ dkey, const uint32_t *__restrict__ dval, const uint2 *__restrict__ rect,
                const unsigned *__restrict__ n_active, int grid_n, int supers_x, int nsup, int chunks,
                const Header *__restrict__ h, const uint32_t *__restrict__ scnt, uint32_t *__restrict__ tab,
                uint32_t *__restrict__ list) {
  extern __shared__ unsigned long long lds_bits[];  // [4][nsup] words, then [4][nsup] counts
  __shared__ uint32_t sstart[kMaxSupers + 1], seg[kMaxSupers + 1];
  if (h->overflow) return;
  super_tables(tab, nsup, sstart, seg);
  if (blockIdx.x == 0)
    for (int s = threadIdx.x; s <= nsup; s += kBlock) {
      tab[kMaxSupers + 1 + s] = sstart[s];
      tab[2 * (kMaxSupers + 1) + s] = seg[s];
    }
  const int w = threadIdx.x >> 6;
  unsigned long long *bits = lds_bits + w * nsup;
  uint32_t *cnt_all = reinterpret_cast<uint32_t *>(lds_bits + 4 * nsup), *cnt = cnt_all + w * nsup;
  for (int s = __lane_id(); s < nsup; s += kWave) {
    bits[s] = 0ull;
    cnt[s] = 0u;
  }
  __builtin_amdgcn_wave_barrier();
  const int nact = n_active ? (int)*n_active : grid_n;
  const int jw = blockIdx.x * kLevel1Chunk + w * (kLevel1Chunk / 4);
  constexpr int rounds = kLevel1Chunk / 4 / kWave;
  for (int r = 0; r < rounds; ++r) {
    uint32_t id, sx0, sy0, nx, area;
    super_rect(dkey, dval, rect, jw + r * kWave + __lane_id(), nact, id, sx0, sy0, nx, area);
    super_round_count(bits, cnt, sx0, sy0, nx, area, supers_x);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nsup; s += kBlock) {  // counts -> first slot of each wave
    const uint32_t a = cnt_all[s], b = cnt_all[nsup + s], c = cnt_all[2 * nsup + s];
    const uint32_t base = sstart[s] + scnt[(int64_t)s * chunks + blockIdx.x];
    cnt_all[s] = base;
    cnt_all[nsup + s] = base + a;
    cnt_all[2 * nsup + s] = base + a + b;
    cnt_all[3 * nsup + s] = base + a + b + c;
  }
  __syncthreads();
  const unsigned long long me = 1ull << __lane_id(), below = lanemask_lt();
  for (int r = 0; r < rounds; ++r) {
    uint32_t id, sx0, sy0, nx, area;
    super_rect(dkey, dval, rect, jw + r * kWave + __lane_id(), nact, id, sx0, sy0, nx, area);
    for (uint32_t k = 0; k < area; ++k) atomicOr(&bits[super_at(k, sx0, sy0, nx, supers_x)], me);
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = 0; k < area; ++k) {
      const uint32_t s = super_at(k, sx0, sy0, nx, supers_x);
      list[cnt[s] + (uint32_t)__popcll(bits[s] & below)] = id;
    }
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = 0; k < area; ++k) {
      const uint32_t s = super_at(k, sx0, sy0, nx, supers_x);
      const unsigned long long b = bits[s];
      if ((b & below) == 0ull) {
        cnt[s] += (uint32_t)__popcll(b);
        bits[s] = 0ull;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Level 2 segment g: super-tile s with seg[s] <= g < seg[s + 1] (segments of
// empty super-tiles have no width), list entries [e0, e1), tile origin.
struct SuperSeg {
  uint32_t e0, e1, tx0, ty0;
  int s;
};

__device__ inline SuperSeg find_segment(uint32_t g, const uint32_t *seg, const uint32_t *sstart,
                                        const uint32_t *slen, int nsup, int supers_x) {
  int lo = 0, hi = nsup;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seg[mid] <= g) lo = mid;
    else hi = mid;
  }
  SuperSeg q;
  q.s = lo;
  q.e0 = sstart[lo] + (g - seg[lo]) * (uint32_t)kSegWave;
  const uint32_t end = sstart[lo] + slen[lo];
  q.e1 = q.e0 + kSegWave < end ? q.e0 + kSegWave : end;
  q.tx0 = (uint32_t)(lo % supers_x) * kSuper;
  q.ty0 = (uint32_t)(lo / supers_x) * kSuper;
  return q;
}

// The tiles of rectangle r inside the super-tile at (tx0, ty0): bit 8 ly + lx.
__device__ inline unsigned long long local_tiles(uint2 r, uint32_t tx0, uint32_t ty0) {
  const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu, y1 = r.y >> 16;
  const uint32_t lx0 = x0 > tx0 ? x0 - tx0 : 0u, ly0 = y0 > ty0 ? y0 - ty0 : 0u;
  const uint32_t lx1 = x1 > tx0 ? (x1 - tx0 < (uint32_t)kSuper ? x1 - tx0 : (uint32_t)kSuper) : 0u;
  const uint32_t ly1 = y1 > ty0 ? (y1 - ty0 < (uint32_t)kSuper ? y1 - ty0 : (uint32_t)kSuper) : 0u;
  if (lx1 <= lx0 || ly1 <= ly0) return 0ull;
  const unsigned long long row = (unsigned long long)((1u << lx1) - (1u << lx0));
  const unsigned long long hi = ly1 >= (uint32_t)kSuper ? ~0ull : (1ull << (8u * ly1)) - 1ull;
  const unsigned long long lo = (1ull << (8u * ly0)) - 1ull;
  return (row * 0x0101010101010101ull) & hi & ~lo;
}

__device__ inline void load_super_tables(const uint32_t *__restrict__ tab, int nsup, uint32_t *slen, uint32_t *sstart,
                                         uint32_t *seg) {
  for (int s = threadIdx.x; s <= nsup; s += blockDim.x) {
    slen[s] = s < nsup ? tab[s] : 0u;
    sstart[s] = tab[kMaxSupers + 1 + s];
    seg[s] = tab[2 * (kMaxSupers + 1) + s];
  }
  __syncthreads();
}

// Level 2 counts: instances of each of the super-tile's 64 tiles in one
// segment (one wave per segment, striding over the segments): the covered
// rectangles go into a per-wave 9x9 difference array, whose 2D prefix gives
// the counts.
__global__ void __launch_bounds__(kBlock)
k_stile_count(const uint32_t *__restrict__ list, const uint2 *__restrict__ rect, const uint32_t *__restrict__ tab,
              int nsup, int supers_x, const Header *__restrict__ h, uint32_t *__restrict__ hist) {
  __shared__ uint32_t slen[kMaxSupers + 1], sstart[kMaxSupers + 1], seg[kMaxSupers + 1];
  __shared__ uint32_t diff[4][(kSuper + 1) * (kSuper + 1)];
  if (h->overflow) return;
  load_super_tables(tab, nsup, slen, sstart, seg);
  const int w = threadIdx.x >> 6, lane = __lane_id();
  const uint32_t total = seg[nsup];
  uint32_t *d = diff[w];
  constexpr int nd = kSuper + 1;
  for (uint32_t g = blockIdx.x * 4u + (uint32_t)w; g < total; g += gridDim.x * 4u) {
    const SuperSeg q = find_segment(g, seg, sstart, slen, nsup, supers_x);
    for (int k = lane; k < nd * nd; k += kWave) d[k] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t e = q.e0 + lane; e < q.e1; e += kWave) {
      const uint2 r = rect[list[e]];
      const uint32_t x0 = r.x & 0xFFFFu, y0 = r.x >> 16, x1 = r.y & 0xFFFFu, y1 = r.y >> 16;
      const uint32_t lx0 = x0 > q.tx0 ? x0 - q.tx0 : 0u, ly0 = y0 > q.ty0 ? y0 - q.ty0 : 0u;
      const uint32_t lx1 = x1 > q.tx0 ? (x1 - q.tx0 < (uint32_t)kSuper ? x1 - q.tx0 : (uint32_t)kSuper) : 0u;
      const uint32_t ly1 = y1 > q.ty0 ? (y1 - q.ty0 < (uint32_t)kSuper ? y1 - q.ty0 : (uint32_t)kSuper) : 0u;
      if (lx1 <= lx0 || ly1 <= ly0) continue;
      atomicAdd(&d[ly0 * nd + lx0], 1u);
      atomicAdd(&d[ly0 * nd + lx1], 0xFFFFFFFFu);
      atomicAdd(&d[ly1 * nd + lx0], 0xFFFFFFFFu);
      atomicAdd(&d[ly1 * nd + lx1], 1u);
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < kSuper) {  // rows
      uint32_t acc = 0;
      for (int x = 0; x < kSuper; ++x) {
        acc += d[lane * nd + x];
        d[lane * nd + x] = acc;
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < kSuper) {  // columns
      uint32_t acc = 0;
      for (int y = 0; y < kSuper; ++y) {
        acc += d[y * nd + lane];
        d[y * nd + lane] = acc;
      }
    }
    __builtin_amdgcn_wave_barrier();
    hist[(int64_t)g * 64 + lane] = d[(lane >> 3) * nd + (lane & 7)];
    __builtin_amdgcn_wave_barrier();
  }
}

// Level 2: per super-tile and tile, exclusive prefix over the super-tile's
// segments of the counts, plus the tile's range start: the first slot of the
// tile's run in every segment (in place).  One kBlock-thread workgroup per
// super-tile: 4 parts of its segments x 64 tiles (a workgroup of the size of
// a compositing one, so that it can start beside a compositing grid).
__global__ void __launch_bounds__(kBlock)
k_stile_scan(uint32_t *__restrict__ hist, const uint32_t *__restrict__ tab, int supers_x, int tiles_x, int tiles_y,
             const uint2 *__restrict__ ranges, const Header *__restrict__ h) {
  constexpr uint32_t kParts = kBlock / 64;
  __shared__ uint32_t part[kParts][64];
  if (h->overflow) return;
  const int s = blockIdx.x;
  const uint32_t g0 = tab[2 * (kMaxSupers + 1) + s], g1 = tab[2 * (kMaxSupers + 1) + s + 1];
  const int tt = threadIdx.x & 63, pp = threadIdx.x >> 6;
  const uint32_t per = (g1 - g0 + kParts - 1u) / kParts;
  const uint32_t a = g0 + (uint32_t)pp * per < g1 ? g0 + (uint32_t)pp * per : g1;
  const uint32_t b = a + per < g1 ? a + per : g1;
  // four counts per step, their reads in flight together (a part spans tens of segments)
  uint32_t *col = hist + tt;
  uint32_t sum = 0, g = a;
  for (; g + 4u <= b; g += 4u) {
    const uint32_t v0 = col[(int64_t)g * 64], v1 = col[(int64_t)(g + 1u) * 64];
    const uint32_t v2 = col[(int64_t)(g + 2u) * 64], v3 = col[(int64_t)(g + 3u) * 64];
    sum += (v0 + v1) + (v2 + v3);
  }
  for (; g < b; ++g) sum += col[(int64_t)g * 64];
  part[pp][tt] = sum;
  __syncthreads();
  const int tx = (s % supers_x) * kSuper + (tt & 7), ty = (s / supers_x) * kSuper + (tt >> 3);
  uint32_t run = (tx < tiles_x && ty < tiles_y) ? ranges[ty * tiles_x + tx].x : 0u;
  for (uint32_t k = 0; k < (uint32_t)pp; ++k) run += part[k][tt];
  for (g = a; g + 4u <= b; g += 4u) {
    const uint32_t v0 = col[(int64_t)g * 64], v1 = col[(int64_t)(g + 1u) * 64];
    const uint32_t v2 = col[(int64_t)(g + 2u) * 64], v3 = col[(int64_t)(g + 3u) * 64];
    col[(int64_t)g * 64] = run;
    run += v0;
    col[(int64_t)(g + 1u) * 64] = run;
    run += v1;
    col[(int64_t)(g + 2u) * 64] = run;
    run += v2;
    col[(int64_t)(g + 3u) * 64] = run;
    run += v3;
  }
  for (; g < b; ++g) {
    const uint32_t v = col[(int64_t)g * 64];
    col[(int64_t)g * 64] = run;
    run += v;
  }
}

// Level 2 scatter, per segment and round of 64 entries: for each of the 64
// tiles one ballot over the lanes whose Gaussian covers it ranks the
// covering lanes; each gets slot base + (covering lanes below), and the
// tile's base (held by lane tt) advances by the ballot's population.  The
// (slot, lane, tile) pairs go to a per-wave LDS queue in tile order, and
// every 64 queued pairs are finished with all lanes busy: the pair's
// wave-block reach mask and one store, consecutive lanes of one tile writing
// consecutive slots.  The queue is drained at the end of each round (the
// stage is then refilled); it never holds more than 63 + 64 pairs.
//
// Reach masks from band intervals.  A wave block is an 8x8 pixel block whose
// origin is a multiple of 8 in both tile shapes, so the super-tile's pixel
// rows fall into tile_h 8-row bands.  When an entry is staged its lane
// computes, for each band its tiles cover, the range of 8-column blocks whose
// pixel-centre box meets the Gaussian's reach ellipse {q' >= log2(1/255) -
// 0.01 - log2 o} -- the criterion block_reach_mask evaluates block by block:
// a block is reached iff the band meets the ellipse and the block's centre
// columns meet the band's x-projection of the ellipse.  That projection ends
// where the ellipse's x-extreme points lie if they fall in the band, else at
// the band edge nearest to them (the ellipse is convex).  The interval is
// widened by a margin for the FP32 evaluation, so the masks stay
// conservative, and kept as a bitmap of the band's tile_w block columns: a
// pair's four mask bits are then bit fields of one or two bitmaps.
//
// A super-tile of 8 x 8 tiles of TW x (256 / TW) pixels has 256 / TW * 8 / 8
// bands of 8 rows and TW 8-column blocks: 16 bands of 16 blocks (16x16
// tiles) or 8 bands of 32 (32x8), each band's bitmap in a word of its width.
// The stage then takes 3,840 bytes per wave, so that a workgroup with its
// super-tile tables fits in the LDS one compositing workgroup leaves (when
// the kernel runs beside a compositing grid on another stream).
template <int TW> struct StileBands;
template <> struct StileBands<16> {
  static constexpr int kBands = 16;
  using Word = uint16_t;
};
template <> struct StileBands<32> {
  static constexpr int kBands = 8;
  using Word = uint32_t;
};

template <int TW>
struct StileStage {
  uint32_t id[kWave];
  // bit c: 8-column block c of the super-tile is reached in this band
  typename StileBands<TW>::Word band[StileBands<TW>::kBands][kWave];
  uint32_t qslot[3 * kWave], qsrc[3 * kWave];  // the queue (2 x 64), then one discard word per lane
};

// The band bitmaps of one entry (its lane's column of sg.band) for the local
// bands [lb0, lb1) of the super-tile whose pixel origin is (sx, sy); ncols =
// TW block columns, so a bitmap fits its word.
template <int TW>
__device__ inline void stage_bands(StileStage<TW> &sg, int lane, float u, float v, float A, float B, float C,
                                   float need, float sx, float sy, int lb0, int lb1, int ncols) {
  const float a = -A;  // > 0: the pre-scaled conic is negative definite
  const float D = 4.0f * A * C - B * B;
  const bool any = need < 0.0f && D > 0.0f && a > 0.0f;
  // x- and y-extent of the ellipse, and the y of its rightmost point (the leftmost is its mirror)
  const float rx = any ? sqrtf(4.0f * C * need / D) : 0.0f;
  const float ry = any ? sqrtf(4.0f * A * need / D) : 0.0f;
  const float yext = any ? -B * rx / (2.0f * C) : 0.0f;
  const float i2a = 0.5f / a;
  const float marg = 0.01f + 1e-4f * (rx + ry);
  for (int lb = lb0; lb < lb1; ++lb) {
    const float yl = sy + (float)(8 * lb) + 0.5f - v, yh = yl + 7.0f;
    uint32_t bits = 0u;
    if (any && yh >= -ry - marg && yl <= ry + marg) {
      const float yr = fminf(fmaxf(yext, yl), yh), yq = fminf(fmaxf(-yext, yl), yh);
      const float dr = fmaxf(B * B * yr * yr + 4.0f * a * (C * yr * yr - need), 0.0f);
      const float dq = fmaxf(B * B * yq * yq + 4.0f * a * (C * yq * yq - need), 0.0f);
      const float xr = u + (B * yr + sqrtf(dr)) * i2a + marg;  // x0(y) = B y / (2a), half width sqrt(disc) / (2a)
      const float xl = u + (B * yq - sqrtf(dq)) * i2a - marg;
      // reached block columns [lo, hi] of the band, clipped to the super-tile
      const float lo = ceilf((xl - 7.5f - sx) * 0.125f), hi = floorf((xr - 0.5f - sx) * 0.125f);
      const int ilo = (int)fminf(fmaxf(lo, 0.0f), (float)ncols);
      const int ihi = (int)fminf(fmaxf(hi, -1.0f), (float)(ncols - 1));
      if (ihi >= ilo) bits = (0xFFFFFFFFu >> (31 - ihi)) & (0xFFFFFFFFu << ilo);
    }
    sg.band[lb][lane] = (typename StileBands<TW>::Word)bits;
  }
}

// Finishes `count` queued (slot, lane, tile) pairs, one per lane: the pair's
// wave-block mask and one store.  Wave block w of a tile at (tx, ty) in the
// super-tile is block column tx * TW / 8 + w % (TW / 8) of band
// ty * (256 / TW) / 8 + w / (TW / 8).
template <int TW>
__device__ inline void stile_flush(const StileStage<TW> &sg, uint32_t head, uint32_t count,
                                   uint32_t *__restrict__ out) {
  const uint32_t lane = __lane_id();
  if (lane < count) {
    const uint32_t pos = (head + lane) & (2 * kWave - 1);
    const uint32_t slot = sg.qslot[pos], src = sg.qsrc[pos];
    const uint32_t l = src & 63u, tt = src >> 8;
    const uint32_t tx = tt & 7u, ty = tt >> 3;
    uint32_t mask;
    if (TW == 16) {  // 16x16: wave blocks 2 x 2, two bands per tile row
      const uint32_t r0 = (uint32_t)sg.band[2 * ty][l], r1 = (uint32_t)sg.band[2 * ty + 1][l];
      mask = ((r0 >> (2 * tx)) & 3u) | (((r1 >> (2 * tx)) & 3u) << 2);
    } else {  // 32x8: wave blocks 4 x 1, one band per tile row
      mask = ((uint32_t)sg.band[ty][l] >> (4 * tx)) & 15u;
    }
    out[slot] = sg.id[l] | (mask << kMaskShift);
  }
  __builtin_amdgcn_wave_barrier();
}

template <int TW>
__global__ void __launch_bounds__(kBlock)
k_stile_scatter(const uint32_t *__restrict__ list, const uint4 *__restrict__ brec, const uint32_t *__restrict__ tab,
                int nsup, int supers_x, const Header *__restrict__ h,
                const uint32_t *__restrict__ hist, uint32_t *__restrict__ out) {
  extern __shared__ uint32_t stab[];  // slen, sstart, seg: nsup + 1 entries each (sized at launch)
  __shared__ StileStage<TW> stage[4];
  if (h->overflow) return;
  uint32_t *slen = stab, *sstart = stab + (nsup + 1), *seg = stab + 2 * (nsup + 1);
  load_super_tables(tab, nsup, slen, sstart, seg);
  const int w = threadIdx.x >> 6, lane = __lane_id();
  StileStage<TW> &sg = stage[w];
  constexpr int TH = kBlock / TW;
  const uint32_t total = seg[nsup];
  for (uint32_t g = blockIdx.x * 4u + (uint32_t)w; g < total; g += gridDim.x * 4u) {
    const SuperSeg q = find_segment(g, seg, sstart, slen, nsup, supers_x);
    uint32_t base = hist[(int64_t)g * 64 + lane];  // lane tt: next slot of the segment's run in tile tt
    for (uint32_t e0 = q.e0; e0 < q.e1; e0 += kWave) {
      const uint32_t e = e0 + lane;
      unsigned long long m = 0ull;
      if (e < q.e1) {
        const uint32_t id = list[e];
        const uint4 b0 = brec[2 * (int64_t)id], b1 = brec[2 * (int64_t)id + 1];
        const uint2 r = make_uint2(b0.x, b0.y);
        m = local_tiles(r, q.tx0, q.ty0);
        sg.id[lane] = id;
        // the entry's tile rows in the super-tile, as 8-row bands
        const uint32_t y0 = r.x >> 16, y1 = r.y >> 16;
        const int ly0 = y0 > q.ty0 ? (int)(y0 - q.ty0) : 0;
        const int ly1 = (int)(y1 - q.ty0) < kSuper ? (int)(y1 - q.ty0) : kSuper;
        stage_bands(sg, lane, __uint_as_float(b0.z), __uint_as_float(b0.w), __uint_as_float(b1.x),
                    __uint_as_float(b1.y), __uint_as_float(b1.z), __uint_as_float(b1.w),
                    (float)(q.tx0 * (uint32_t)TW), (float)(q.ty0 * (uint32_t)TH), ly0 * TH / 8, ly1 * TH / 8, TW);
      }
      __builtin_amdgcn_wave_barrier();
      uint32_t head = 0, tail = 0;  // wave-uniform queue positions
      // one pass per 32-bit half of the tile mask (tiles 0..31, then 32..63)
      auto tiles_of = [&](uint32_t word, int tt0) {
        for (int t = 0; t < 32; ++t) {
          const int tt = tt0 + t;
          const bool mine = __builtin_amdgcn_ubfe(word, (uint32_t)t, 1u) != 0u;
          const unsigned long long b = __builtin_amdgcn_ballot_w64(mine);
          if (b == 0ull) continue;
          const uint32_t bt = __builtin_amdgcn_readlane(base, tt);
          const uint32_t nb = (uint32_t)__popcll(b);
          // a covering lane queues its pair at tail + (covering lanes below
          // it); the others write their own discard word (no branch)
          const uint32_t rank =
              __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
          const uint32_t pos = mine ? ((tail + rank) & (2 * kWave - 1)) : 2 * kWave + (uint32_t)lane;
          sg.qslot[pos] = bt + rank;
          sg.qsrc[pos] = (uint32_t)lane | ((uint32_t)tt << 8);
          base = lane == tt ? bt + nb : base;  // lane tt's base advances past the tile's run
          tail += nb;
          __builtin_amdgcn_wave_barrier();
          if (tail - head >= (uint32_t)kWave) {
            stile_flush<TW>(sg, head, kWave, out);
            head += kWave;
          }
        }
      };
      tiles_of((uint32_t)m, 0);
      tiles_of((uint32_t)(m >> 32), 32);
      if (tail != head) stile_flush<TW>(sg, head, tail - head, out);
    }
  }
}

void launch_super_scatter(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                          int grid_n, int tiles_x, int tiles_y, int tile_w, int tile_h, const uint4 *brec,
                          const uint2 *ranges, const Header *h,
                          uint32_t *scnt, uint32_t *tab, uint32_t *list, uint32_t *hist, int64_t cap,
                          uint32_t *out, hipStream_t st) {
  if (grid_n <= 0) return;
  const int supers_x = (tiles_x + kSuper - 1) / kSuper, supers_y = (tiles_y + kSuper - 1) / kSuper;
  const int nsup = supers_x * supers_y;
  const int chunks = (int)ceil_div(grid_n, kLevel1Chunk);
  const size_t lds = (size_t)nsup * 4 * (sizeof(unsigned long long) + sizeof(uint32_t));
  k_super_count<<<chunks, kBlock, lds, st>>>(dkey, dval, rect, n_active, grid_n, supers_x, nsup, chunks, h, scnt);
  k_super_scan<<<nsup, kBlock, 0, st>>>(scnt, chunks, h, tab);
  k_super_scatter<<<chunks, kBlock, lds, st>>>(dkey, dval, rect, n_active, grid_n, supers_x, nsup, chunks, h, scnt,
                                               tab, list);
  // level 2 strides over at most cap / kSegWave + nsup segments
  const int64_t segs = cap / kSegWave + nsup + 1;
  const int64_t blocks = ceil_div(segs, 4) < 4096 ? ceil_div(segs, 4) : 4096;
  k_stile_count<<<(unsigned)blocks, kBlock, 0, st>>>(list, rect, tab, nsup, supers_x, h, hist);
  k_stile_scan<<<nsup, kBlock, 0, st>>>(hist, tab, supers_x, tiles_x, tiles_y, ranges, h);
  const size_t tables = 3 * sizeof(uint32_t) * (size_t)(nsup + 1);
  if (tile_w == 16)
    k_stile_scatter<16><<<(unsigned)blocks, kBlock, tables, st>>>(list, brec, tab, nsup, supers_x, h, hist, out);
  else  // 32 x 8, the other tile shape
    k_stile_scatter<32><<<(unsigned)blocks, kBlock, tables, st>>>(list, brec, tab, nsup, supers_x, h, hist, out);
}

bool launch_tile_ranges(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                        int grid_n, int tiles_x, int tiles_y, Header *h, uint32_t *tdiff, uint32_t *tcnt,
                        uint32_t *tstart, unsigned long long *parts, uint2 *ranges, hipStream_t st,
                        bool tdiff_zeroed, uint32_t *tile_order) {
  const int tiles = tiles_x * tiles_y;
  const int64_t ne = (int64_t)(tiles_x + 1) * (tiles_y + 1);
  if (!tdiff_zeroed) k_zero_u32<<<(unsigned)ceil_div(ne, kBlock), kBlock, 0, st>>>(tdiff, ne);
  if (grid_n > 0) {
    // enough workgroups to cover the machine, few enough to keep the LDS flushes cheap
    const int64_t per = ne <= kDiffLds ? (grid_n / 512 > 1024 ? grid_n / 512 : 1024) : 1024;
    const int blocks = (int)ceil_div(grid_n, per);
    const size_t lds = ne <= kDiffLds ? sizeof(uint32_t) * (size_t)ne : 0;
    k_tile_diff<<<blocks, kBlock, lds, st>>>(dkey, dval, rect, n_active, grid_n, tiles_x, tiles_y, tdiff);
  }
  if (ne <= kDiffLds) {
    k_tile_ranges_lds<<<1, kBlock, sizeof(uint32_t) * (size_t)ne, st>>>(tdiff, tiles_x, tiles_y, h, ranges,
                                                                         tile_order);
    return tile_order != nullptr;
  }
  k_tile_prefix<<<1, 1024, 0, st>>>(tdiff, tiles_x, tiles_y, tcnt);
  launch_scan_u32(tcnt, tstart, tiles, parts, &h->instances, st);
  k_ranges_from_counts<<<(unsigned)ceil_div(tiles, kBlock), kBlock, 0, st>>>(tcnt, tstart, tiles, h, ranges);
  return false;
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

// Present count of every state (one workgroup per state) from the
// (packet, layer) histogram.
__global__ void __launch_bounds__(kBlock)
k_state_counts(const uint8_t *__restrict__ codes, const uint32_t *__restrict__ hist, int P,
               uint32_t *__restrict__ cnt) {
  const int w = blockIdx.x;
  uint32_t c = 0;
  for (int p = threadIdx.x; p < P; p += kBlock) {
    const int code = codes[(int64_t)w * P + p];
    const uint4 h = *reinterpret_cast<const uint4 *>(hist + (int64_t)p * kPlStride);
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
// so that the S states of a group have similar list-walk depths.  Launched
// with kBlock threads up to kBlock states (the size of a compositing
// workgroup, so that it can start beside a compositing grid), else 1024.
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
  k_state_rank<<<1, num_states <= kBlock ? kBlock : 1024, sizeof(uint32_t) * num_states, st>>>(cnt, num_states,
                                                                                               order);
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
