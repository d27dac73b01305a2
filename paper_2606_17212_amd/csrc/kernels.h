// Host-side launchers of the renderer's kernels (internal to libdgs.so).
#pragma once

#include "common.h"

namespace dgs {

// geometry.hip
void launch_geometry(const SceneArgs &s, const CamArgs &c, const TileArgs &t, const uint32_t *list,
                     const unsigned *n_active, int grid_n, float4 *rec0, float4 *rec1, float4 *rec2,
                     uint2 *rect, uint2 *pbox, uint32_t *dkey, uint32_t *dval, hipStream_t st);
void launch_geometry_bwd(const SceneArgs &s, const CamArgs &c, const float *g2d, float *g_mean,
                         float *g_ls, float *g_quat, float *g_logit, float *g_color, float *g_temporal,
                         hipStream_t st);

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
void launch_clear_header(Header *h, unsigned long long capacity, hipStream_t st);
void launch_count(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                  int grid_n, uint32_t *cnt, hipStream_t st);
void launch_emit(const uint32_t *dval, const uint2 *rect, const uint32_t *off, const uint32_t *cnt,
                 const unsigned *n_active, int grid_n, int tiles_x, int tile_w, int tile_h, const float4 *rec0,
                 const float4 *rec1, const uint2 *pbox, Header *h, uint32_t *tkey, uint32_t *tval,
                 hipStream_t st);
// Per-tile [start, end) of the tile-sorted instances, from the Gaussians'
// tile rectangles (the same instances emission writes); empty after an overflow.
void launch_tile_ranges(const uint32_t *dkey, const uint32_t *dval, const uint2 *rect, const unsigned *n_active,
                        int grid_n, int tiles_x, int tiles_y, const Header *h, uint32_t *tdiff, uint32_t *tcnt,
                        uint32_t *tstart, unsigned long long *parts, uint2 *ranges, hipStream_t st);
void launch_visbits(const uint8_t *codes, const uint32_t *order, int num_states, int P, int S,
                    uint32_t *visbits, hipStream_t st);
void launch_plhist(const uint16_t *packet_layer, int n, int P, uint32_t *hist, hipStream_t st);
constexpr int kMaxOrderedStates = 16384;  // states ranked by present count per composite call
void launch_state_order(const uint8_t *codes, const uint32_t *hist, int num_states, int P, uint32_t *cnt,
                        uint32_t *order, hipStream_t st);
void launch_tile_order(const uint2 *ranges, int tiles, uint32_t *order, hipStream_t st);
void launch_present_flags(const uint8_t *codes_row, const uint16_t *packet_layer, int n, int P,
                          uint32_t *flags, hipStream_t st);
void launch_present_scatter(const uint32_t *flags, const uint32_t *off, int n, uint32_t *list,
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
};
// mode 0: images, 1: per-tile squared error for PSNR, 2: work counters only.
// launch 0: automatic, 1: persistent, 2: grid.
int launch_composite(const CompositeArgs &a, int S, int tile_w, int tile_h, int mode, int launch,
                     hipStream_t st);
void launch_zero_queues(unsigned int *queues, hipStream_t st);
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

}  // namespace dgs
