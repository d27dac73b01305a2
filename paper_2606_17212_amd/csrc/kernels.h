// Host-side launchers of the renderer's kernels (internal to libdgs.so).
#pragma once

#include "common.h"

namespace dgs {

// geometry.hip
// plhist (or null): zeroed [P][kPlStride] Gaussian counts per (packet, layer), added
// to by the same launch (every Gaussian once; not with a list).
void launch_geometry(const SceneArgs &s, const CamArgs &c, const TileArgs &t, const uint32_t *list,
                     const unsigned *n_active, int grid_n, float4 *rec0, float4 *rec1, float4 *rec2,
                     uint2 *rect, uint2 *pbox, uint4 *brec, uint32_t *dkey, uint32_t *dval, hipStream_t st,
                     uint32_t *plhist = nullptr);
void launch_geometry_bwd(const SceneArgs &s, const CamArgs &c, const float *g2d, float *g_mean,
                         float *g_ls, float *g_quat, float *g_logit, float *g_color, float *g_temporal,
                         float *g_refine, hipStream_t st);

// sort.hip: exclusive scan of u32 values (total written as u64 when non-null)
// and stable LSD radix sort of (u32 key, u32 value) pairs.
void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, unsigned long long *parts,
                     unsigned long long *total, hipStream_t st);
// Sorts bits [begin_bit, end_bit) of the keys.  Count = *count_dev clamped to
// max_count when count_dev is non-null, else max_count.  Ping-pongs between
// (k0,v0) and (k1,v1); returns 0 if the result is in (k0,v0), 1 otherwise.
// last_pass_keys = false: the final pass writes values only (keys not needed).
int launch_radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const void *count_dev,
                      int count_is_u64, int64_t max_count, int begin_bit, int end_bit, uint32_t *hist,
                      unsigned long long *parts, hipStream_t st, bool last_pass_keys = true);

// binning.hip
// Resets the header; also zeroes za[0..na) and zb[0..nb) when given.
void launch_clear_header(Header *h, unsigned long long capacity, hipStream_t st, uint32_t *za = nullptr,
                         int64_t na = 0, uint32_t *zb = nullptr, int64_t nb = 0);
void launch_count(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                  int grid_n, uint32_t *cnt, hipStream_t st);
void launch_emit(const uint32_t *dval, const uint2 *rect, const uint32_t *off, const uint32_t *cnt,
                 const unsigned *n_active, int grid_n, int tiles_x, int tile_w, int tile_h, const float4 *rec0,
                 const float4 *rec1, const uint2 *pbox, Header *h, uint32_t *tkey, uint32_t *tval,
                 hipStream_t st);
// Per-tile [start, end) of the tile-sorted instances, from the Gaussians'
// tile rectangles (the same instances emission writes); empty after an overflow.
// The same launch writes the instance count to h->instances and sets
// h->overflow when it exceeds h->capacity.
// tdiff_zeroed: the (tiles_x + 1) (tiles_y + 1) difference array is already
// zero.  tile_order (or null): when the grid fits LDS the same launch also
// writes the tiles by decreasing list length; returns whether it did.
bool launch_tile_ranges(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                        int grid_n, int tiles_x, int tiles_y, Header *h, uint32_t *tdiff, uint32_t *tcnt,
                        uint32_t *tstart, unsigned long long *parts, uint2 *ranges, hipStream_t st,
                        bool tdiff_zeroed = false, uint32_t *tile_order = nullptr);
bool tile_ranges_in_lds(int tiles_x, int tiles_y);
// Two-level stable scatter of the instances into their tiles' ranges (needs
// the ranges and the overflow flag of launch_tile_ranges; super_path grids):
// scnt, tab, list and hist are workspace sections (super_cnt, super_tab, and
// cap-sized tkey0 / tkey1), out the tile-sorted values.
void launch_super_scatter(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                          int grid_n, int tiles_x, int tiles_y, int tile_w, int tile_h, const uint4 *brec,
                          const uint2 *ranges, const Header *h,
                          uint32_t *scnt, uint32_t *tab, uint32_t *list, uint32_t *hist, int64_t cap,
                          uint32_t *out, hipStream_t st);
void launch_visbits(const uint8_t *codes, const uint32_t *order, int num_states, int P, int S, bool exact,
                    uint32_t *visbits, hipStream_t st);
constexpr int kMaxOrderedStates = 16384;  // states ranked by present count per composite call
void launch_state_order(const uint8_t *codes, const uint32_t *hist, int num_states, int P, uint32_t *cnt,
                        uint32_t *order, hipStream_t st);
void launch_tile_order(const uint2 *ranges, int tiles, uint32_t *order, hipStream_t st);
void launch_present_flags(const uint8_t *codes_row, const uint16_t *packet_layer, int n, int P,
                          uint32_t *flags, hipStream_t st);
void launch_present_scatter(const uint32_t *flags, const uint32_t *off, int n, const uint8_t *codes_row,
                            const uint16_t *packet_layer, bool refined, uint32_t *list,
                            const unsigned long long *total, Header *h, hipStream_t st);
void launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);
void launch_fill_u64(unsigned long long *p, int n, hipStream_t st);  // zero n <= 64 counters

// composite.hip
struct CompositeArgs {
  const float4 *rec0, *rec1, *rec2;
  const uint32_t *vals;        // tile-sorted values: Gaussian id | wave-block reach mask << 28
  const uint2 *ranges;         // per tile [start, end)
  const uint32_t *visbits;     // [groups][P*4] state bits, or null (every entry visible, S = 1)
  const uint32_t *tile_order;  // tiles by decreasing list length
  const uint32_t *state_order; // group slot -> state index, or null (identity)
  int P4;                      // P * 4
  int num_states, width, height, tiles_x, tiles_y, groups;
  float bg[3];
  float *image;                // [W][H][Wd][3]
  float *tfinal;               // [W][H][Wd] or null
  const float *reference;      // [H][Wd][3] (PSNR mode)
  float *psnr_part;            // [W][tiles] (PSNR mode)
  int state_offset;            // first state index of this launch's images
  int launch_states;           // states composited by this launch
  unsigned long long *counters;  // [4] (count mode)
  unsigned int *queues;        // [8] per-XCD work counters (persistent launch)
  struct {                     // pair mode (counterfactual utility)
    const unsigned long long *item_total;  // work items wanted (device)
    uint64_t item_capacity;                // patches available
    int num_contexts;
    const uint32_t *item_base;     // [J + 1] first work item of each context
    const int32_t *context_group;  // [J]
    const uint32_t *group_base;    // [G + 1] first region tile of each group
    const uint32_t *region_tiles;  // tiles of each group's region, by group
    const unsigned long long *bundle_total;  // compositing work items over all bundles (device)
    const uint32_t *bundle_base;   // [J] first compositing item of the bundle context j starts
    const uint32_t *bad;           // [J] context without work items
  } pair;
};
// mode 0: images, 1: per-tile squared error for PSNR, 2: work counters only.
// launch 0: automatic, 1: persistent, 2: grid.  lds_batch: list entries staged
// per batch (128, 256 or 512; variants exist for S >= 4 in modes 0 and 1, 256
// is used otherwise).
int launch_composite(const CompositeArgs &a, int S, int tile_w, int tile_h, int mode, int launch, int lds_batch,
                     hipStream_t st);
void launch_zero_queues(unsigned int *queues, hipStream_t st);
// Pair mode: composites every (context, region tile) work item for the
// context and the context plus its group into a.image patches
// [item][2][tile_w * tile_h][3]; a.visbits holds [J][P*4] two-bit words.
// Up to four consecutive contexts of one group ("a bundle") are composited
// together at one tile as one 8-state group.
int launch_composite_pairs(const CompositeArgs &a, int tile_w, int tile_h, int workgroups, hipStream_t st);
// How launch_composite runs image mode for `groups` state groups (host only).
struct CompositePlan {
  bool persistent;
  int64_t workgroups;  // workgroups launched
  int64_t items;       // (tile, state group) work items
  int lds_batch;       // list entries staged per LDS batch by the chosen variant
};
int plan_composite(int S, int tile_w, int tile_h, int tiles, int groups, int launch, int lds_batch,
                   CompositePlan *out);
void launch_psnr_finalize(const float *psnr_part, int num_states, int tiles, int64_t pixels,
                          float *psnr, hipStream_t st);

struct CompositeBwdArgs {
  const float4 *rec0, *rec1, *rec2;
  const uint32_t *vals;
  const uint2 *ranges;
  const uint32_t *visbits;
  const uint32_t *tile_order;
  const uint32_t *state_order;
  int P4;
  int num_states, width, height, tiles_x, tiles_y, groups;
  const float *image, *grad_image;
  float *g2d;                  // [9][n]: d/d(u, v, A', B', C', log2 o, r, g, b)
  int n;
};
int launch_composite_bwd(const CompositeBwdArgs &a, int S, int tile_w, int tile_h, hipStream_t st);

// utility.hip: counterfactual render utility, distortion, risk adjustment
struct UtilHeader {
  unsigned long long regions;       // region tiles over all groups
  unsigned long long items;         // work items over all contexts
  unsigned long long bundle_items;  // compositing work items over all bundles
  unsigned int bad_group;      // 1: a group's packet is out of range; 2: two groups name one (packet, layer)
  unsigned int bad_context;    // 1: a context lacks its group's packet at exactly the group's layer
  unsigned int queue[8];
};

constexpr int kMaxRiskValues = 4096;  // contexts per group in dgs_risk_adjusted

struct UtilLayout {
  size_t hdr, pl2g, core, region, wcount, wprefix, region_tiles, group_base, icount, item_base, bad, pvis, parts,
      partial, patches, bcount, bbase, total;
  int64_t words;
};

inline UtilLayout make_util_layout(int64_t P, int64_t tiles, int64_t G, int64_t J, int64_t cap) {
  UtilLayout L{};
  L.words = ceil_div(tiles, 32);
  const int64_t gw = G * L.words;
  const int64_t scan_n = gw > J ? gw : J;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + (bytes > 0 ? bytes : 1)); return at; };
  L.hdr = take(sizeof(UtilHeader));
  L.pl2g = take(4 * P * 4);
  L.core = take(4 * gw);
  L.region = take(4 * gw);
  L.wcount = take(4 * gw);
  L.wprefix = take(4 * gw);
  L.region_tiles = take(4 * G * tiles);
  L.group_base = take(4 * (G + 1));
  L.icount = take(4 * J);
  L.item_base = take(4 * J);
  L.bad = take(4 * J);
  L.pvis = take(4 * J * P * 4);
  L.parts = take(8 * (ceil_div(scan_n, kScanTile) + 1));
  L.partial = take(4 * cap);
  L.patches = take((size_t)4 * cap * 2 * kBlock * 3);
  L.bcount = take(4 * J);
  L.bbase = take(4 * J);
  L.total = o;
  return L;
}

struct UtilArgs {
  UtilHeader *hdr;
  int *pl2g;
  uint32_t *core, *region, *wcount, *wprefix, *region_tiles, *group_base, *icount, *item_base, *bad, *pvis;
  uint32_t *bcount, *bbase;  // work items of the bundle a context starts (0 if none), and their prefix
  unsigned long long *parts;
  float *partial, *patches, *delta;
  const unsigned long long *item_total;  // &hdr->items
  unsigned int *queue;                   // hdr->queue
  uint64_t item_capacity;
  int num_contexts, words, tiles_x, tiles_y, width, height;
  int refined;  // the scene has refinement levels: records are (Gaussian, delivered depth)
  const int32_t *context_group;
  const float *reference;
  float lambda;
};

// A context starts a compositing bundle unless it continues the previous
// context's: same group, both with work items, and not at a multiple of four
// (so a bundle holds one to four contexts of one group).
__device__ inline bool bundle_start(const int32_t *context_group, const uint32_t *bad, int j) {
  return j == 0 || (j & 3) == 0 || context_group[j] != context_group[j - 1] || bad[j] != 0u || bad[j - 1] != 0u;
}

void launch_clear_util_header(UtilHeader *h, hipStream_t st);
// Group tables, core tiles, regions (core dilated by rx, ry tiles) and the
// region tile lists, from the rectangles of the last binning.
void launch_group_setup(const UtilArgs &u, const uint16_t *group_pl, int G, int P, const float4 *rec0,
                        const uint2 *rect, int n, int rx, int ry, hipStream_t st);
// Pair delivery bits and work items per context (total in hdr->items).
void launch_pair_setup(const UtilArgs &u, const uint8_t *codes, const uint16_t *group_pl, int G, int P,
                       hipStream_t st);
// Per-item SSIM / squared-error differences, then Delta per context.
int launch_pair_ssim(const UtilArgs &u, int tile_w, int tile_h, int workgroups, hipStream_t st);
void launch_distortion(const float *images, int num_images, int width, int height, const float *reference,
                       float lambda, double *part, float *d, hipStream_t st);
void launch_risk_adjusted(const float *values, const int32_t *offsets, int G, float alpha, float beta, float q,
                          float *out, hipStream_t st);

// sampler.hip: delivery states drawn on the device (layout of dgs_channel)
struct SamplerChannel {
  float p_gb, p_bg, loss_good, loss_bad, p_start_bad;
  int32_t deadline;
};
void launch_sample_states(const SamplerChannel *channels, int num_states, int P, int L, uint64_t seed,
                          uint8_t *codes, hipStream_t st);

}  // namespace dgs
