// Shared definitions of the HIP renderer library (device helpers, kernel
// parameter blocks, workspace layout).  Internal to libdgs.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dgs {

constexpr int kWave = 64;
constexpr int kBlock = 256;         // every kernel runs 256-thread workgroups (4 waves)
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;
constexpr float kQCut = 11.1f;      // >= 2 ln 255: outside the rectangle alpha < 1/255
constexpr float kDilation = 0.3f;
constexpr float kShC0 = 0.28209479177387814f;
constexpr float kShC1 = 0.4886025119029199f;
// alpha = min(0.99, 2^q') with q' = A' dx^2 + B' dx dy + C' dy^2 + log2(o), where
// (A', B', C') = (kConicA A, kConicB B, kConicA C) pre-scale the conic (A, B, C):
// 2^q' = o exp(-(A dx^2 + 2 B dx dy + C dy^2) / 2).
constexpr float kConicA = -0.72134752044448170f;  // -log2(e) / 2
constexpr float kConicB = -1.4426950408889634f;   // -log2(e)
constexpr float kQSkip = -7.9943534368588578f;    // log2(1/255): alpha < 1/255 <=> q' < kQSkip
// Tile-sorted values: Gaussian id in bits 0..27, bit 28 + w set when the
// Gaussian can reach alpha >= 1/255 somewhere in wave block w of that tile.
constexpr uint32_t kIdMask = 0x0FFFFFFFu;
constexpr int kMaskShift = 28;
constexpr int kMaxGaussians = 0x0FFFFFFF;

// Origin of wave w's 8x8 pixel block inside a TW-wide tile (16x16: 2x2
// blocks; 32x8: 4x1 blocks).
__host__ __device__ inline int wave_block_x0(int w, int tw) { return (w * 8) % tw; }
__host__ __device__ inline int wave_block_y0(int w, int tw) { return ((w * 8) / tw) * 8; }

// Largest value of the exponent A' X^2 + B' X Y + C' Y^2 (negative definite)
// over the box X in [xl, xh], Y in [yl, yh]: 0 when the box holds the origin.
// Otherwise the maximum lies on an edge facing the origin (from any other
// boundary point the segment towards the origin enters the box and the
// concave exponent increases along it), at most one X edge and one Y edge,
// at the clamped 1D maximiser X* = B Y ia, Y* = B X ic with ia = -1/(2 A),
// ic = -1/(2 C).  An inexact maximiser only lowers the value found by a
// second-order amount, which the caller's margin absorbs.
__device__ inline float box_max_exponent(float A, float B, float C, float ia, float ic, float xl, float xh,
                                         float yl, float yh) {
  const bool inx = xl <= 0.0f && xh >= 0.0f, iny = yl <= 0.0f && yh >= 0.0f;
  if (inx && iny) return 0.0f;
  float best = -INFINITY;
  if (!inx) {
    const float X = xl > 0.0f ? xl : xh;
    const float Y = fminf(fmaxf(B * X * ic, yl), yh);
    best = fmaf(A * X, X, fmaf(B * X, Y, C * Y * Y));
  }
  if (!iny) {
    const float Y = yl > 0.0f ? yl : yh;
    const float X = fminf(fmaxf(B * Y * ia, xl), xh);
    best = fmaxf(best, fmaf(A * X, X, fmaf(B * X, Y, C * Y * Y)));
  }
  return best;
}

__device__ inline bool box_reaches(float A, float B, float C, float ia, float ic, float xl, float xh, float yl,
                                   float yh, float need) {
  return box_max_exponent(A, B, C, ia, ic, xl, xh, yl, yh) >= need;
}

// Whether every pixel centre of a box reaches `need`: the exponent is concave,
// so its minimum over the box is at a corner.
__device__ inline bool box_all_reach(float A, float B, float C, float xl, float xh, float yl, float yh, float need) {
  const float q00 = fmaf(A * xl, xl, fmaf(B * xl, yl, C * yl * yl));
  const float q01 = fmaf(A * xl, xl, fmaf(B * xl, yh, C * yh * yh));
  const float q10 = fmaf(A * xh, xh, fmaf(B * xh, yl, C * yl * yl));
  const float q11 = fmaf(A * xh, xh, fmaf(B * xh, yh, C * yh * yh));
  return fminf(fminf(q00, q01), fminf(q10, q11)) >= need;
}

// Scene parameters passed by value to kernels.
struct SceneArgs {
  int n, rank, sh_degree, num_contexts, num_packets;
  const float *mean, *log_scale, *quat, *opacity_logit, *color, *temporal;
  const uint16_t *packet_layer;
  const float *affine;
  const float *refine;  // [3][refine_rows][n] refinement levels, or null
  int refine_rows;
  float basis[4];
};

struct CamArgs {
  float R[9];
  float t[3];
  float fx, fy, cx, cy, near_z;
  int width, height;
  float campos[3];  // camera centre in world space (-R^T t)
};

struct TileArgs {
  int tile_w, tile_h, tiles_x, tiles_y;
};

// Device-side counters at the start of the workspace.
struct Header {
  unsigned long long instances;   // tile instances of the last binning
  unsigned long long capacity;    // capacity that binning was given
  unsigned int overflow;          // 1 if instances > capacity
  unsigned int n_active;          // Gaussians entering the last binning
  unsigned int pad[10];
};

// Workspace layout (byte offsets, each 256-aligned).
struct Layout {
  size_t header;
  size_t rec0, rec1, rec2;   // float4 [n] each: (u, v, log2 o, packet_layer bits), (A', B', C', depth), (r, g, b, 0)
  size_t rect;               // uint2 [n]: (x0 | y0 << 16, x1 | y1 << 16) in tiles
  size_t pbox;               // uint2 [n]: the same rectangle in pixels
  size_t brec;               // uint4 [2n]: (rect, u, v) then (A', B', C', reach bound) -- what level 2 reads per entry
  size_t dkey0, dkey1, dval0, dval1;  // depth sort ping-pong [n]
  size_t cnt;                // u32 [n]: instance counts, then offsets (sorted order)
  size_t present;            // u32 [n]: per-state compaction flags / list
  size_t part;               // u64 scan partials
  size_t tkey0, tkey1, tval0, tval1;  // tile sort ping-pong [cap]
  size_t hist;               // u32 radix histograms
  size_t ranges;             // uint2 [tiles]
  size_t tdiff;              // u32 [(tiles_y+1)(tiles_x+1)]: 2D difference array of tile coverage
  size_t super_cnt;          // u32 [supers][level-1 chunks]: counts, then first slots (two-level scatter)
  size_t super_tab;          // u32 [3][kMaxSupers + 1]: list length, list start, first segment per super-tile
  size_t tcnt, tstart;       // u32 [tiles]: instances per tile and their exclusive scan
  size_t grad2d;             // f32 [9][n]
  size_t plhist;             // u32 [P][kPlStride]: Gaussians per (packet, layer), a packet's four layers per row
  size_t tile_order;         // u32 [tiles]: tiles by decreasing list length
  size_t state_cnt;          // u32 [max_states]: present Gaussians per state
  size_t state_order;        // u32 [max_states]: states by increasing present count
  size_t visbits;            // u32 [max_states][P*4]
  size_t psnr_part;          // f32 [max_states][tiles]
  size_t queues;             // u32 [8]: per-XCD work queues of the persistent compositing launch
  size_t total;
  int64_t n, cap, tiles, max_states, P;
  int64_t sort_blocks;       // blocks of the largest radix pass
  int64_t scan_parts;        // entries of the partials buffer
};

// Row of the (packet, layer) histogram: a packet's four counts at the start
// of their own 128-byte line, so that the projection's atomic adds spread
// over as many lines as there are packets.
constexpr int kPlStride = 32;
constexpr int kDiffLds = 12288;   // tile-coverage entries held in LDS (48 KB): (tiles_x + 1) (tiles_y + 1)
// Two-level instance scatter: super-tiles of kSuper x kSuper tiles (one bit
// per tile in a u64), at most kMaxSupers of them; level 1 takes kLevel1Chunk
// depth-ordered Gaussians per workgroup, level 2 kSegWave list entries per wave.
constexpr int kSuper = 8;
constexpr int kMaxSupers = 1024;
constexpr int kLevel1Chunk = 256;
constexpr int kSegWave = 128;
inline int64_t supers_of(int64_t tiles_x, int64_t tiles_y) {
  return ((tiles_x + kSuper - 1) / kSuper) * ((tiles_y + kSuper - 1) / kSuper);
}
inline bool super_path(int64_t tiles_x, int64_t tiles_y) { return supers_of(tiles_x, tiles_y) <= kMaxSupers; }
constexpr int kSortIpt = 16;
constexpr int kSortTile = kBlock * kSortIpt;  // 4096 keys per radix workgroup (the largest tile)
// Keys per radix workgroup for a sort of `count` keys: smaller tiles for
// small sorts, so that up to 256 workgroups share each pass (whose digit
// offsets the scatter kernel then forms from the raw histograms itself).
inline int sort_tile_for(int64_t count) {
  return count <= (int64_t)256 * 1024 ? 1024 : (count <= (int64_t)256 * 2048 ? 2048 : kSortTile);
}
inline int64_t sort_blocks_for(int64_t count) {
  const int64_t c = count > 0 ? count : 1;
  return (c + sort_tile_for(c) - 1) / sort_tile_for(c);
}
constexpr int kScanTile = kBlock * 16;        // 4096 values per scan workgroup

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline Layout make_layout(int64_t n, int64_t P, int64_t tiles_x, int64_t tiles_y, int64_t max_states,
                          int64_t cap) {
  const int64_t tiles = tiles_x * tiles_y;
  Layout L{};
  L.n = n; L.cap = cap; L.tiles = tiles; L.max_states = max_states; L.P = P;
  int64_t nn = n > 0 ? n : 1;
  int64_t cc = cap > 0 ? cap : 1;
  int64_t big = nn > cc ? nn : cc;
  (void)big;
  L.sort_blocks = sort_blocks_for(nn) > sort_blocks_for(cc) ? sort_blocks_for(nn) : sort_blocks_for(cc);
  int64_t hist_entries = 256 * L.sort_blocks;
  int64_t scan_max = hist_entries > nn ? hist_entries : nn;
  if (tiles > scan_max) scan_max = tiles;  // the scan over tiles of the ranges for large grids
  L.scan_parts = ceil_div(scan_max, kScanTile) + 1;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  L.header = take(sizeof(Header));
  L.rec0 = take(16 * nn);
  L.rec1 = take(16 * nn);
  L.rec2 = take(16 * nn);
  L.rect = take(8 * nn);
  L.pbox = take(8 * nn);
  L.brec = take(32 * nn);
  L.dkey0 = take(4 * nn);
  L.dkey1 = take(4 * nn);
  L.dval0 = take(4 * nn);
  L.dval1 = take(4 * nn);
  L.cnt = take(4 * nn);
  L.present = take(4 * nn);
  L.part = take(8 * L.scan_parts);
  L.tkey0 = take(4 * cc);  // two-level scatter: the super-tile lists (at most cap entries)
  {
    // two-level scatter: per level-2 segment 64 tile counts, then first slots; a super-tile of
    // len entries has ceil(len / kSegWave) segments, so at most cap / kSegWave + supers in all
    const int64_t segs = super_path(tiles_x, tiles_y) ? cc / kSegWave + supers_of(tiles_x, tiles_y) + 1 : 0;
    L.tkey1 = take(4 * cc > 4 * 64 * segs ? 4 * cc : 4 * 64 * segs);
  }
  L.tval0 = take(4 * cc);
  L.tval1 = take(4 * cc);
  L.hist = take(4 * hist_entries);
  L.ranges = take(8 * (tiles > 0 ? tiles : 1));
  L.tdiff = take(4 * (tiles_x + 1) * (tiles_y + 1));
  {
    const bool sp = super_path(tiles_x, tiles_y);
    L.super_cnt = take(sp ? 4 * supers_of(tiles_x, tiles_y) * ceil_div(nn, kLevel1Chunk) : 4);
    L.super_tab = take(4 * 3 * (kMaxSupers + 1));
  }
  L.tcnt = take(4 * (tiles > 0 ? tiles : 1));
  L.tstart = take(4 * (tiles > 0 ? tiles : 1));
  L.grad2d = take(4 * 9 * nn);
  L.plhist = take(4 * P * kPlStride);
  L.tile_order = take(4 * (tiles > 0 ? tiles : 1));
  L.state_cnt = take(4 * (max_states > 0 ? max_states : 1));
  L.state_order = take(4 * (max_states > 0 ? max_states : 1));
  L.visbits = take(4 * (max_states > 0 ? max_states : 1) * P * 4);
  L.psnr_part = take(4 * (max_states > 0 ? max_states : 1) * (tiles > 0 ? tiles : 1));
  L.queues = take(4 * 8);
  L.total = o;
  return L;
}

template <typename T>
inline T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ---------------------------------------------------------------- wave helpers

__device__ inline unsigned long long lanemask_lt() {
  unsigned lane = __lane_id();
  return (1ull << lane) - 1ull;
}

__device__ inline unsigned long long lanemask_gt() {
  unsigned lane = __lane_id();
  return lane == 63 ? 0ull : (~0ull << (lane + 1));
}

template <typename T>
__device__ inline T wave_incl_scan(T x) {
  const unsigned lane = __lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d, kWave);
    if (lane >= (unsigned)d) x += y;
  }
  return x;
}

}  // namespace dgs
