/*
 * dgs.h -- C ABI of the batched partial-delivery Gaussian renderer for
 * AMD MI355X (gfx950).
 *
 * The library renders one dynamic Gaussian scene (Sec. 3 of the paper:
 * clustered Gaussians, Eq. (1) affine + low-rank temporal motion, one base and
 * three refinement groups per cluster) under many incomplete delivery states
 * at once (Sec. 6: states of shape [W, N, .] rasterised in one call, FP32
 * rasterisation, batched evaluation bit-equivalent to serial evaluation).  A
 * delivery state is a cluster/context packet mask with a delivered prefix
 * depth, formed after dependency enforcement (Sec. 4).
 *
 * Conventions for every entry point:
 *  - Pointers marked "device" are HIP device pointers; "host" are host
 *    pointers.  The caller owns all memory: scene, codes, images, gradients
 *    and the workspace.  The library allocates nothing on the render path.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call except
 *    dgs_count_instances, dgs_check, dgs_utility_count and
 *    dgs_utility_check is asynchronous on that stream:
 *    device buffers must stay valid until the stream's work completes.
 *  - Return value: a dgs_status.  Arguments are validated before any HIP call;
 *    on failure nothing is launched and dgs_last_error() (thread-local)
 *    describes the problem.  No exception crosses the ABI and nothing aborts.
 *  - Floating point: FP32 throughout the device path.  Depth keys, culling
 *    and tile rectangles follow a fixed FP32 operation order, so binning and
 *    sort keys are reproducible bit for bit; a state's image is bit-identical
 *    whether it is rendered alone (dgs_render_per_state) or batched
 *    (dgs_render), with either tile shape.
 *  - Graph capture: the calls that synchronise (dgs_count_instances,
 *    dgs_check, dgs_utility_count, dgs_utility_check, dgs_objective_check)
 *    return DGS_ERR_INVALID_ARG, before any launch, on a stream that is
 *    being captured; every other call only enqueues work and may be captured.
 *  - Concurrency: all device state of a call lives in its workspace and its
 *    outputs (dgs_render_noalloc's in the library's one static array, see
 *    there).  Calls on different workspaces may run at the same time on
 *    different streams; calls on one workspace must be ordered by the caller
 *    (one stream, or events).  Renders of successive batches on two or three
 *    streams, each with its own workspace, overlap one batch's binning with
 *    the compositing of the batches before it.
 *
 * Plan / forward / poll: sizing is dgs_workspace_bytes plus the one
 * synchronising count dgs_count_instances; the forward is dgs_render (or
 * dgs_bin followed by any number of dgs_composite calls); dgs_check polls for
 * overflow and asynchronous errors.  There is no context object: tuning is an
 * explicit dgs_tuning argument and graph capture belongs to the caller.
 */
#ifndef DGS_H
#define DGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGS_ABI_VERSION 3

typedef enum {
  DGS_OK = 0,
  DGS_ERR_INVALID_ARG = 1, /* bad pointer, size or shape; nothing launched */
  DGS_ERR_WORKSPACE = 2,   /* workspace smaller than dgs_workspace_bytes() */
  DGS_ERR_OVERFLOW = 3,    /* tile instances exceeded the capacity (dgs_check) */
  DGS_ERR_HIP = 4,         /* a HIP runtime call failed (message in dgs_last_error) */
  DGS_ERR_UNSUPPORTED = 5  /* tuning outside the compiled variants */
} dgs_status;

/*
 * Scene: structure of arrays, FP32, component-major [k][n] (row k holds
 * component k of every Gaussian).  All pointers are device pointers.
 *   mean          [3][n]   canonical means (mu-bar of Eq. (1))
 *   log_scale     [3][n]   per-axis log standard deviation
 *   quat          [4][n]   rotation quaternion (w, x, y, z), any non-zero norm
 *   opacity_logit [n]      opacity = sigmoid(logit)
 *   color         [3][n]   RGB (sh_degree 0) or [12][n] degree-1 real SH,
 *                          row = coefficient * 3 + channel (sh_degree 1)
 *   temporal      [3*rank][n]  per-Gaussian temporal coefficients q_{i,r} of
 *                          Eq. (1), row = r * 3 + axis
 *   packet_layer  [n]      (packet << 2) | layer, packet = cluster * K + context,
 *                          layer 0..3 (base + three refinements, Sec. 3)
 *   cluster_affine [C][12] per-cluster 3x4 affine A_{c,t} of Eq. (1) at the
 *                          render time, row-major, or NULL for the identity
 *   refine        [3][rows][n]  attribute refinement levels 1..3 (Sec. 3:
 *                          scale, rotation, opacity and colour are a base
 *                          plus three refinements; the position carries
 *                          residual levels on top of the deformation), or
 *                          NULL.  rows = 14 (sh_degree 0) or 23 (sh_degree 1):
 *                          position residual at the render time 3, log-scale
 *                          3, quaternion 4, opacity logit 1, colour 3 or 12
 *                          (same row order as `color`).
 * Limits: 0 <= n < 2^28 (4n < 2^28 with refine); rank 0..4; sh_degree 0 or 1;
 * 1 <= C*K <= 16384.
 *
 * With refine, a Gaussian of packet p delivered to depth d (code d+1, present
 * when its layer <= d) is drawn with base + level 1 + ... + level d of every
 * attribute (each sum rounded once, in that order) and its position residual
 * (level 1 + ... + level d, summed from zero) added after the deformation.
 * The renderer projects one record per (Gaussian, depth) - 4n records, size
 * the workspace for n_records = 4n - and each state draws the record of the
 * depth it delivers.  dgs_backward also returns the levels' gradients
 * (dgs_scene_grad.refine); the utility calls take such scenes (adding group
 * (p, l) moves packet p from depth l - 1 to depth l), and so does
 * dgs_render_per_state (each state's delivered records).
 */
typedef struct {
  int32_t n;
  int32_t rank;
  int32_t sh_degree;
  int32_t num_clusters;
  int32_t num_contexts;
  const float *mean;
  const float *log_scale;
  const float *quat;
  const float *opacity_logit;
  const float *color;
  const float *temporal;
  const uint16_t *packet_layer;
  const float *cluster_affine;
  const float *refine;
} dgs_scene;

/* Pinhole camera (host struct): world -> camera rotation R_cw (row-major) and
 * translation t_cw; OpenCV frame (x right, y down, z forward); focal lengths
 * and principal point in pixels; pixel (x, y) has its centre at (x+0.5, y+0.5).
 * Gaussians with camera depth <= near_z are culled.  1 <= width, height <= 16384. */
typedef struct {
  float R_cw[9];
  float t_cw[3];
  float fx, fy, cx, cy, near_z;
  int32_t width, height;
} dgs_camera;

/* Delivery states.  codes: device [num_states][C*K] uint8; code 0 = packet
 * absent, d+1 = prefix depth d (layers 0..d delivered).  Gaussian (packet p,
 * layer l) is present in state w iff l < codes[w][p]; codes above 4 act as 4.
 * basis: host b_r(t) for r < rank (the shared temporal basis of Eq. (1) at
 * the render time).  background: host RGB composited behind every pixel. */
typedef struct {
  int32_t num_states;
  const uint8_t *codes;
  float basis[4];
  float background[3];
} dgs_states;

/* Launch shape.  tile_w x tile_h in {16x16, 32x8} (0,0 = 16x16);
 * states_per_group in {1,2,4,8,16,32} (0 = 16): states composited together
 * by one workgroup, sharing each splat's alpha evaluation.
 * flags: how the batched compositing is launched; results are identical.
 *   DGS_TUNE_GRID: one workgroup per (tile, state group) work item.
 *   DGS_TUNE_PERSISTENT: one workgroup per resident slot, draining per-XCD
 *     work queues (heavy tiles first, then stealing from other XCDs).
 *   0: automatic - persistent when there are at least 32 work items per
 *     resident slot, or groups of 16 or more states and at least 4 work items
 *     per resident slot; else grid.  Setting both bits is DGS_ERR_INVALID_ARG. */
#define DGS_TUNE_PERSISTENT 1
#define DGS_TUNE_GRID 2
typedef struct {
  int32_t tile_w;
  int32_t tile_h;
  int32_t states_per_group;
  int32_t flags;
  int32_t lds_batch;  /* list entries staged in LDS per batch: 128, 256 or 512 (0 = 256);
                         used for states_per_group >= 4 in image and PSNR mode */
} dgs_tuning;

/* Parameter gradients, device pointers with the scene's shapes; overwritten.
 * refine: [3][rows][n] gradients of the refinement levels (required when the
 * scene has them, else ignored): level j's gradient sums the gradients of the
 * Gaussian's records at depths >= j; the base parameters' sum all its records. */
typedef struct {
  float *mean;
  float *log_scale;
  float *quat;
  float *opacity_logit;
  float *color;
  float *temporal;
  float *refine;
} dgs_scene_grad;

int dgs_abi_version(void);
const char *dgs_status_string(int status);
/* Message describing the last failure on the calling thread ("" if none). */
const char *dgs_last_error(void);

/*
 * Bytes of device workspace needed by the calls below for a scene of n
 * projected records (n Gaussians, or 4n with refinement levels) and num_packets = C*K packets seen by `cam` with tuning `tun`,
 * at most max_states states per call, and room for instance_capacity
 * (tile, Gaussian) instances.  Returns 0 on invalid arguments.
 * The workspace is caller-owned device memory, at least 256-byte aligned.
 */
size_t dgs_workspace_bytes(int32_t n, int32_t num_packets, const dgs_camera *cam,
                           const dgs_tuning *tun, int32_t max_states,
                           int64_t instance_capacity);

/*
 * Projects every Gaussian (masks ignored) and counts its tile instances; the
 * total is the capacity a render of any subset of the scene needs.
 * SYNCHRONISES the stream and writes the count to *instances (host).
 * ws may be sized with instance_capacity = 0.
 */
int dgs_count_instances(const dgs_scene *scene, const dgs_camera *cam,
                        const dgs_states *states, const dgs_tuning *tun, void *ws,
                        size_t ws_bytes, int64_t *instances, void *stream);

/*
 * Batched render (the hot path; Sec. 6: the states of one scene are
 * rasterised in one call, in FP32).  Deformation (Eq. (1)) and projection of all
 * Gaussians, tile binning and the (tile, depth, index) sort run once; then
 * every state is composited front to back from the shared per-tile lists,
 * skipping Gaussians its codes do not deliver (the cluster-layer masks of
 * Sec. 4).
 *   image  device [W][height][width][3] FP32, colour + T_final * background
 *   tfinal device [W][height][width] transmittance after the last
 *          composited Gaussian, or NULL
 * instance_capacity: as passed to dgs_workspace_bytes; if the scene needs
 * more instances the output is undefined and dgs_check reports
 * DGS_ERR_OVERFLOW.  Work on the stream only: safe to capture in a HIP graph.
 * The workspace keeps the sorted lists for a following dgs_backward.
 */
int dgs_render(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
               const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t instance_capacity,
               float *image, float *tfinal, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dgs_render
 * with its workspace in a static device array of the library instead of a
 * caller-owned buffer.  Same arguments, outputs and kernels as dgs_render
 * (the images are bit-identical), without ws / ws_bytes.
 *   instances  device int64 [1] or NULL: receives the tile instances the
 *              scene needs (as dgs_check reports them); more than
 *              instance_capacity means the images are undefined (overflow).
 * Limit: the call's workspace (dgs_workspace_bytes of the same arguments)
 * must fit DGS_NOALLOC_SCRATCH_BYTES, else DGS_ERR_WORKSPACE before any HIP
 * call.  The array is allocated with the library's device code on each GPU
 * it runs on and held until the process ends; this call allocates and frees
 * nothing and does not synchronise.  All calls on one GPU share that GPU's
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (concurrent streams or threads) race and must be serialised by the caller.
 * dgs_backward and dgs_check cannot name this array.
 */
#define DGS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int dgs_render_noalloc(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                       const dgs_tuning *tun, int64_t instance_capacity, float *image, float *tfinal,
                       int64_t *instances, void *stream);

/*
 * The two halves of dgs_render (Sec. 6: one scene and time shared by every
 * state of the batch).  dgs_bin runs the shared part -- deformation,
 * projection, depth sort, tile binning and the per-tile lists -- for the
 * scene and camera (states->codes is not read; basis is).  dgs_composite then
 * composites every state in `states` from those lists; it may be called any
 * number of times after one dgs_bin (e.g. a sweep over many state batches of
 * one scene and time), with the same scene, camera, tuning, workspace and
 * capacity.  Outputs as for dgs_render.
 */
int dgs_bin(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
            const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t instance_capacity,
            void *stream);
int dgs_composite(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                  const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t instance_capacity,
                  float *image, float *tfinal, void *stream);

/*
 * PSNR of every state against `reference` from the lists of the last dgs_bin
 * (as dgs_render_psnr, without the binning).
 */
int dgs_composite_psnr(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                       const dgs_tuning *tun, void *ws, size_t ws_bytes,
                       int64_t instance_capacity, const float *reference, float *psnr,
                       void *stream);

/*
 * How dgs_composite launches the batched compositing of `num_states` states
 * with this camera and tuning (host query; the device that will run it must be
 * current, for the occupancy query).  Outputs (host): *states_per_group = S
 * used; *persistent = 1 for the persistent launch, 0 for the grid launch;
 * *workgroups = workgroups launched; *work_items = (tile, state group) work
 * items; *lds_batch = list entries staged per LDS batch by the variant that
 * runs (the tuning's, or 256 where S < 4).  Returns DGS_OK, DGS_ERR_INVALID_ARG, DGS_ERR_UNSUPPORTED or
 * DGS_ERR_HIP.
 */
int dgs_composite_launch(const dgs_camera *cam, const dgs_tuning *tun, int32_t num_states, int32_t *states_per_group,
                         int32_t *persistent, int64_t *workgroups, int64_t *work_items, int32_t *lds_batch);

/*
 * Work counters of dgs_composite for the same arguments, nothing rendered:
 * counters (device, 4 x u64, overwritten) = { alpha evaluations: (pixel,
 * list entry, state group) triples where some delivered state of the group is
 * still compositing that pixel; blends: (pixel, state, Gaussian) triples
 * composited, i.e. present Gaussians with alpha >= 1/255 before the stop;
 * wave evaluations: (64-pixel block, entry, group) triples evaluated; wave
 * misses: those of them where no pixel of the block reached alpha >= 1/255 }.
 */
int dgs_composite_stats(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                        const dgs_tuning *tun, void *ws, size_t ws_bytes,
                        int64_t instance_capacity, unsigned long long *counters, void *stream);

/*
 * Plain per-state render (baseline; with a synchronisation after each call it
 * is the serial evaluation Sec. 6 compares against, whose results the paper
 * states batched evaluation reproduces bit for bit): for each state in turn, compacts the
 * delivered Gaussians, projects, bins, sorts and composites only them.
 * Same outputs, bit-identical to dgs_render's.  tun->states_per_group is
 * ignored.  instance_capacity from dgs_count_instances covers every state.
 */
int dgs_render_per_state(const dgs_scene *scene, const dgs_camera *cam,
                         const dgs_states *states, const dgs_tuning *tun, void *ws,
                         size_t ws_bytes, int64_t instance_capacity, float *image,
                         float *tfinal, void *stream);

/*
 * Batched render reduced on device to one PSNR per state against `reference`
 * (the per-state image-space evaluation behind Sec. 5's utilities and
 * Sec. 6's utility-state throughput)
 * (device [height][width][3]): PSNR = 10 log10(1 / max(MSE, 1e-10)), MSE over
 * every pixel and channel, accumulated from per-tile FP32 partial sums in
 * FP64.  No image is written.  psnr: device [W] FP32.
 */
int dgs_render_psnr(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                    const dgs_tuning *tun, void *ws, size_t ws_bytes,
                    int64_t instance_capacity, const float *reference, float *psnr,
                    void *stream);

/*
 * Backward of dgs_render (Sec. 4 and Sec. 6: training renders and
 * differentiates the batched states; gradients of Eq. (1)'s parameters,
 * scale, rotation, opacity and colour).  Must follow a dgs_render with the same arguments
 * and the same, untouched workspace (its sorted lists are reused; per tile the
 * compositing is recomputed front to back, no per-pixel lists are stored).
 *   image      device [W][H][Wd][3]: the forward's output
 *   grad_image device [W][H][Wd][3]: dL/d image
 *   grad       parameter gradients summed over all states (overwritten).
 * Gradients are accumulated with FP32 atomics: not bitwise reproducible.
 * tun->states_per_group above 8 is clamped to 8 here.
 */
int dgs_backward(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                 const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t instance_capacity,
                 const float *image, const float *grad_image, const dgs_scene_grad *grad,
                 void *stream);

/*
 * SYNCHRONISES the stream, then reports the instance count of the last
 * binning in ws (*instances, may be NULL) and DGS_ERR_OVERFLOW if it exceeded
 * the capacity that call was given; also returns DGS_ERR_HIP for a pending
 * asynchronous HIP error.
 */
int dgs_check(void *ws, size_t ws_bytes, int64_t *instances, void *stream);

/*
 * Byte offsets, inside a workspace laid out for the given sizes, of the
 * intermediate results a render leaves behind (for inspection and tests):
 *   rec0/rec1/rec2  float4 [n] per record (Gaussian i, or 4i + d for depth d
 *                   with refinement levels): (u, v, log2 opacity,
 *                   packet_layer bits - the layer field holds d with
 *                   refinement levels), (conic A, B, C scaled by -log2(e)/2,
 *                   -log2(e), -log2(e)/2, FP32 camera depth), (r, g, b, 0);
 *                   only records that entered the last binning are written
 *   rect            uint2 [n]: (x0 | y0 << 16, x1 | y1 << 16), half-open tiles
 *   ranges          uint2 [tiles]: [start, end) of each tile's list
 *   sorted_ids      u32 [capacity]: record ids in (tile, depth, id) order in
 *                   bits 0..27; bit 28 + b is set when the Gaussian can reach
 *                   alpha >= 1/255 in the tile's 8x8 pixel block b (blocks in
 *                   row-major order: 2x2 for 16x16 tiles, 4x1 for 32x8)
 * Returns DGS_OK or DGS_ERR_INVALID_ARG.  Host-only; launches nothing.
 */
typedef struct {
  uint64_t rec0, rec1, rec2, rect, ranges, sorted_ids;
  int32_t tiles_x, tiles_y;
} dgs_workspace_view;

int dgs_workspace_sections(int32_t n, int32_t num_packets, const dgs_camera *cam,
                           const dgs_tuning *tun, int32_t max_states, int64_t instance_capacity,
                           dgs_workspace_view *out);

/* ---------------------------------------------------------------------------
 * Counterfactual render utility (Sec. 5).
 *
 * A completion group g = (packet p, layer l) is a packet's refinement layer;
 * its marginal utility in a context m (Eq. (3)) is
 *     Delta_g(m) = D(I, R(m)) - D(I, R(m u g)),
 * where m holds packet p at prefix depth exactly l (layers 0..l-1 delivered,
 * code l) and m u g holds it at depth l + 1 (code l + 1).  D is the
 * distortion the paper fixes for its objective (Sec. 4):
 *     D(I, X) = MSE(I, X) + lambda (1 - SSIM(I, X))     (lambda = 0.20 there)
 * with MSE and SSIM averaged over every pixel and channel; SSIM uses the
 * 11 x 11 Gaussian window (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, and zero
 * padding outside the image.  The two renders differ only near g's Gaussians,
 * so each context composites only the tiles of g's Gaussians plus a ring of
 * tiles 10 pixels deep, both states at once.
 * ------------------------------------------------------------------------- */

/*
 * Bytes of the utility workspace (caller-owned, 256-byte aligned, separate
 * from the render workspace) for num_groups groups, num_contexts contexts
 * and item_capacity work items (one item = one context x one tile of its
 * group's region; dgs_utility_count gives the number needed).  0 for invalid
 * arguments.  Host-only.
 */
size_t dgs_utility_workspace_bytes(int32_t num_packets, const dgs_camera *cam, const dgs_tuning *tun,
                                   int32_t num_groups, int32_t num_contexts, int64_t item_capacity);

/*
 * Work items dgs_utility needs for these groups and contexts (synchronises).
 * Arguments as for dgs_utility; the scene, camera, tuning and render
 * workspace must be those of the last dgs_bin.  *items (host) = work items.
 * Returns DGS_ERR_INVALID_ARG when a group names a packet outside the scene,
 * two groups name the same (packet, layer), or a context does not hold its
 * group's packet at exactly the group's layer.
 */
int dgs_utility_count(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *contexts,
                      const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t instance_capacity,
                      const int32_t *context_group, const uint16_t *group_pl, int32_t num_groups,
                      void *uws, size_t uws_bytes, int64_t *items, void *stream);

/*
 * Eq. (3) for every context, from the per-tile lists of the last dgs_bin of
 * this scene, camera and tuning in `ws`.
 *   contexts       codes u8 [J][P] (device) = the contexts m; basis and
 *                  background as for dgs_render
 *   context_group  i32 [J] (device): the group of each context
 *   group_pl       u16 [G] (device): (packet << 2) | layer of each group
 *   reference      f32 [H][W][3] (device): the image I
 *   lambda         weight of (1 - SSIM) in D
 *   uws            utility workspace of dgs_utility_workspace_bytes(...,
 *                  item_capacity)
 *   delta          f32 [J] (device, written): Delta_g(m); NaN for an invalid
 *                  context and for every context after an item overflow
 * Asynchronous; dgs_utility_check reports invalid groups or contexts and
 * overflow.
 */
int dgs_utility(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *contexts,
                const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t instance_capacity,
                const int32_t *context_group, const uint16_t *group_pl, int32_t num_groups,
                const float *reference, float lambda, void *uws, size_t uws_bytes,
                int64_t item_capacity, float *delta, void *stream);

/*
 * Status of the last dgs_utility on `uws` (synchronises): DGS_OK,
 * DGS_ERR_INVALID_ARG (as for dgs_utility_count) or DGS_ERR_OVERFLOW (more
 * work items than item_capacity).  *items (host, may be NULL) = items needed.
 */
int dgs_utility_check(void *uws, size_t uws_bytes, int64_t item_capacity, int64_t *items, void *stream);

/*
 * D(I, X) = MSE + lambda (1 - SSIM) of each of num_images images X
 * [num_images][H][W][3] (device) against reference I [H][W][3] (device), as
 * defined above; d f32 [num_images] (device, written).  scratch (device,
 * 8-byte aligned) of dgs_distortion_scratch_bytes() bytes.  Asynchronous.
 */
size_t dgs_distortion_scratch_bytes(int32_t num_images, int32_t width, int32_t height);
int dgs_distortion(const float *images, int32_t num_images, int32_t width, int32_t height,
                   const float *reference, float lambda, void *scratch, size_t scratch_bytes, float *d,
                   void *stream);

/*
 * Risk-adjusted utility, Eq. (4), per group:
 *     ((1 - alpha) E[Delta] + alpha Q_q(Delta)) / (1 + beta Std(Delta))
 * over the values of group k = values[offsets[k] .. offsets[k+1]) (device
 * f32 / i32 [G+1]; 1..4096 values per group).  The quantile interpolates
 * linearly between order statistics at position (n - 1) q; Std is the
 * population standard deviation.  out f32 [G][4] (device, written) = (mean,
 * quantile, std, risk-adjusted); all NaN for a group with a NaN value or a
 * count outside 1..4096.  The paper uses alpha = 0.25, beta = 0.05,
 * q = 0.10.  Asynchronous.
 */
int dgs_risk_adjusted(const float *values, const int32_t *offsets, int32_t num_groups, float alpha,
                      float beta, float quantile, float *out, void *stream);

/* ---------------------------------------------------------------------------
 * Delivery states drawn on the device (Sec. 4: a training world samples
 * erasures from an IID and a Gilbert-Elliott burst process; dependencies are
 * enforced after delivery and become cluster-layer masks).
 *
 * Every (packet p, layer l) is one datagram, sent layer-major: slot
 * s = l * num_packets + p.  A world's channel is a two-state Markov chain
 * over the slots: the datagram of slot s is erased with the current state's
 * loss probability, then the chain moves (good -> bad with p_gb, bad -> good
 * with p_bg); the first state is bad with probability p_start_bad (IID
 * erasure: p_gb = p_start_bad = 0).  Slots >= deadline arrive too late
 * (deadline < 0: no deadline).  Layer l of packet p is usable when layers
 * 0..l all arrived, so code[w][p] = number of leading arrived layers (the
 * code convention of dgs_states).
 *
 * Draws: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed (low
 * word first).  Counter (s / 2, w, 0x44475331, 0) gives the (erasure,
 * transition) draws of slot s from outputs (0, 1) for even s and (2, 3) for
 * odd s; counter (0xffffffff, w, 0x44475331, 0) output 0 draws the first
 * state.  An event of probability p happens when its 32-bit draw is below
 * floor(p * 2^32) (never for p <= 0, always for p >= 1).  World w's codes
 * depend only on (seed, w, its channel), not on num_states.
 * ------------------------------------------------------------------------- */
typedef struct {
  float p_gb;         /* good -> bad per datagram */
  float p_bg;         /* bad -> good per datagram */
  float loss_good;    /* erasure probability in the good state */
  float loss_bad;     /* erasure probability in the bad state */
  float p_start_bad;  /* probability that the first datagram meets the bad state */
  int32_t deadline;   /* slots that arrive before the playout deadline; < 0: all */
} dgs_channel;

/*
 *   channels  dgs_channel [num_states] (device)
 *   codes     u8 [num_states][num_packets] (device, written)
 * num_packets in 1..16384, num_layers in 1..4.  Asynchronous.  Returns
 * DGS_OK or DGS_ERR_INVALID_ARG.
 */
int dgs_sample_states(const dgs_channel *channels, int32_t num_states, int32_t num_packets, int32_t num_layers,
                      uint64_t seed, uint8_t *codes, void *stream);

/* ---------------------------------------------------------------------------
 * Packet-conditioned rendering objective (Sec. 4, Eq. (2)) and its gradient
 * with respect to the rendered images, for one training batch:
 *
 *   L = E[D] + lambda_c CVaR_alpha(D) + lambda_t F + lambda_m M + lambda_a D_anchor
 *
 * D_k = MSE + lambda_ssim (1 - SSIM) of image k against targets[target_of[k]]
 * (SSIM: 11x11 Gaussian window, sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, zero
 * padding, mean over pixels and channels).  Roles (device int32 lists of image
 * indices):
 *   expect   [num_expect]     partial delivery states: E[D] is their mean D;
 *                             CVaR_alpha the mean of the worst alpha fraction
 *                             of their D (the largest floor(alpha n) count
 *                             fully, the next the remainder, over alpha n;
 *                             ties by list position)
 *   anchor   [num_anchor]     complete-prefix states (mean D)
 *   mono     [num_mono][2]    (a, b): state b grows a's prefix; M = mean of
 *                             max(0, D_b - D_a)
 *   temporal [num_temporal][2] (a, b): one world at two times; F = mean over
 *                             pairs of the mean of ((I_b - I_a) - (G_b - G_a))^2
 * The rate proxy R of Eq. (2) has weight 0 in the configuration the paper
 * locks and does not depend on the images; it is not part of L here.
 * Paper's weights: lambda_ssim 0.20, lambda_c 0.30, alpha 0.05, lambda_t 0.10,
 * lambda_m 2.0, lambda_a 0.50.
 */
typedef struct {
  float lambda_ssim, lambda_c, alpha, lambda_t, lambda_m, lambda_a;
} dgs_objective_weights;

/* Scratch bytes for dgs_objective (0 on invalid sizes): about 36 B per image
 * pixel plus per-block partial sums.  num_images <= 65536, num_temporal <= 65536. */
size_t dgs_objective_scratch_bytes(int32_t num_images, int32_t width, int32_t height, int32_t num_temporal);

/*
 * images [num_images][height][width][3] FP32 and targets [num_targets][...]
 * (device); target_of [num_images] int32 (device).  Outputs (device):
 *   loss       float [6]: L, E[D], CVaR, F, M, anchor D (required)
 *   distortion float [num_images]: D per image, or NULL
 *   grad       float [num_images][height][width][3]: dL/d images, or NULL
 *              (the gradient of every image, zero for images in no role)
 * scratch: caller-owned device memory of dgs_objective_scratch_bytes, 256-byte
 * aligned, overwritten.  Limits: num_expect <= 4096, the other lists <= 65536;
 * weights finite and >= 0, alpha in (0, 1].  Asynchronous, deterministic
 * (every sum in a fixed order).  An index out of range in a device list
 * makes the loss NaN and is reported by dgs_objective_check.  Returns DGS_OK,
 * DGS_ERR_INVALID_ARG, DGS_ERR_WORKSPACE or DGS_ERR_HIP.
 */
int dgs_objective(const float *images, int32_t num_images, int32_t width, int32_t height, const float *targets,
                  int32_t num_targets, const int32_t *target_of, const int32_t *expect, int32_t num_expect,
                  const int32_t *anchor, int32_t num_anchor, const int32_t *mono, int32_t num_mono,
                  const int32_t *temporal, int32_t num_temporal, const dgs_objective_weights *weights,
                  float *loss, float *distortion, float *grad, void *scratch, size_t scratch_bytes,
                  void *stream);

/* SYNCHRONISES the stream; DGS_ERR_INVALID_ARG if the last dgs_objective on
 * this scratch met an index out of range, else DGS_OK. */
int dgs_objective_check(void *scratch, size_t scratch_bytes, void *stream);

/*
 * Plain photometric L1 loss, for training on a target without the Eq. (2)
 * terms (whose distortion D, Sec. 4, is MSE + SSIM): the mean over all
 * num_images * height * width * 3 elements of |images - targets[target_of[k]]|
 * (target_of device int32 [num_images], or NULL: every image against target 0).
 * dgs_l1_loss writes the loss (device float [1]; 0 for an empty batch).  Its
 * scratch (device, 256-byte aligned, dgs_l1_scratch_bytes, 0 on invalid
 * sizes) starts with the flag dgs_objective_check reads: a target index
 * outside 0..num_targets-1 makes the loss NaN, and dgs_objective_check then
 * returns DGS_ERR_INVALID_ARG.  The sum is formed in FP64 partials in a fixed
 * order (reproducible bit for bit).
 * dgs_l1_loss_grad writes grad [num_images][height][width][3] =
 * dloss * sign(image - target) / (num_images * height * width * 3), sign(0) = 0,
 * with dloss a device float [1] (the upstream gradient of the loss) or NULL
 * for 1; NaN for an image whose target index is out of range.  Both are
 * asynchronous on `stream`; num_images <= 65535.  Returns DGS_OK,
 * DGS_ERR_INVALID_ARG, DGS_ERR_WORKSPACE or DGS_ERR_HIP.
 */
size_t dgs_l1_scratch_bytes(int32_t num_images, int32_t width, int32_t height);
int dgs_l1_loss(const float *images, int32_t num_images, int32_t width, int32_t height, const float *targets,
                int32_t num_targets, const int32_t *target_of, float *loss, void *scratch, size_t scratch_bytes,
                void *stream);
int dgs_l1_loss_grad(const float *images, int32_t num_images, int32_t width, int32_t height, const float *targets,
                     int32_t num_targets, const int32_t *target_of, const float *dloss, float *grad, void *stream);


/* ---------------------------------------------------------------------------
 * Measured roofs (for reporting kernels against the machine as well as
 * against its published peaks; nothing on the render path uses these).
 *
 * dgs_probe_copy: copies `bytes` (a multiple of 16, both pointers 16-byte
 * aligned device pointers) from src to dst with 16-byte loads and stores;
 * reads and writes each byte once, so bytes moved = 2 * bytes.
 * dgs_probe_valu: DGS_PROBE_THREADS threads (8 waves per SIMD on 256 CUs),
 * each running 8 independent chains of `iterations` (1 .. 2^24) steps:
 * kind 0 an FP32 fused multiply-add per step (2 FLOPs), kind 1 one hardware
 * base-2 exponential per step; out: device float [DGS_PROBE_THREADS] (one
 * value per thread, written so the work is not optimised away).
 * Both asynchronous on `stream`; DGS_ERR_INVALID_ARG for bad arguments,
 * DGS_ERR_HIP for a failed launch.
 */
#define DGS_PROBE_THREADS 524288
int dgs_probe_copy(const void *src, void *dst, size_t bytes, void *stream);
int dgs_probe_valu(int32_t kind, int64_t iterations, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DGS_H */
