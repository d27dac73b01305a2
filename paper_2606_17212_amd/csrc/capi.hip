// C ABI of the renderer: argument validation, workspace layout and the launch
// sequence of each entry point.  Declarations and contracts: include/dgs.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "../../include/dgs.h"
#include "common.h"
#include "kernels.h"
#include "objective.h"

using namespace dgs;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_check(const char *where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DGS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
  return DGS_OK;
}

// Entry points that copy a header to the host and wait for it cannot be part
// of a captured graph: they refuse a stream that is being captured (before
// any launch), instead of leaving the capture invalid.
int refuse_capture(hipStream_t st, const char *what) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DGS_ERR_HIP, "%s: capture status of the stream: %s", what, hipGetErrorString(e));
  }
  if (cs != hipStreamCaptureStatusNone)
    return fail(DGS_ERR_INVALID_ARG, "%s synchronises with the host and cannot run under graph capture", what);
  return DGS_OK;
}

struct Tiling {
  int tw, th, tiles_x, tiles_y, tiles, tile_bits;
};

int check_tuning(const dgs_camera *cam, const dgs_tuning *tun, Tiling *t) {
  int tw = 16, th = 16;
  if (tun && (tun->tile_w || tun->tile_h)) {
    tw = tun->tile_w;
    th = tun->tile_h;
  }
  if (!((tw == 16 && th == 16) || (tw == 32 && th == 8)))
    return fail(DGS_ERR_UNSUPPORTED, "tile shape %dx%d not supported (16x16 or 32x8)", tw, th);
  if (tun && (tun->flags & ~(DGS_TUNE_PERSISTENT | DGS_TUNE_GRID)) != 0)
    return fail(DGS_ERR_INVALID_ARG, "unknown tuning flags");
  if (tun && (tun->flags & DGS_TUNE_PERSISTENT) && (tun->flags & DGS_TUNE_GRID))
    return fail(DGS_ERR_INVALID_ARG, "tuning flags: persistent and grid are exclusive");
  if (tun && tun->lds_batch != 0 && tun->lds_batch != 128 && tun->lds_batch != 256 && tun->lds_batch != 512)
    return fail(DGS_ERR_UNSUPPORTED, "lds_batch %d not supported (128, 256 or 512)", tun->lds_batch);
  t->tw = tw;
  t->th = th;
  t->tiles_x = (cam->width + tw - 1) / tw;
  t->tiles_y = (cam->height + th - 1) / th;
  t->tiles = t->tiles_x * t->tiles_y;
  int bits = 1;
  while ((1 << bits) < t->tiles) ++bits;
  t->tile_bits = bits;
  return DGS_OK;
}

int check_camera(const dgs_camera *cam) {
  if (!cam) return fail(DGS_ERR_INVALID_ARG, "camera is NULL");
  if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
    return fail(DGS_ERR_INVALID_ARG, "camera size %dx%d outside 1..16384", cam->width, cam->height);
  if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f) || !isfinite(cam->fx) || !isfinite(cam->fy))
    return fail(DGS_ERR_INVALID_ARG, "focal lengths must be positive and finite");
  for (int k = 0; k < 9; ++k)
    if (!isfinite(cam->R_cw[k])) return fail(DGS_ERR_INVALID_ARG, "R_cw not finite");
  for (int k = 0; k < 3; ++k)
    if (!isfinite(cam->t_cw[k])) return fail(DGS_ERR_INVALID_ARG, "t_cw not finite");
  if (!isfinite(cam->cx) || !isfinite(cam->cy) || !isfinite(cam->near_z))
    return fail(DGS_ERR_INVALID_ARG, "principal point / near plane not finite");
  // a non-positive near plane would let depths at or behind the camera through
  if (!(cam->near_z > 0.0f)) return fail(DGS_ERR_INVALID_ARG, "near_z %g must be positive", (double)cam->near_z);
  return DGS_OK;
}

int check_scene(const dgs_scene *s) {
  if (!s) return fail(DGS_ERR_INVALID_ARG, "scene is NULL");
  if (s->n < 0 || s->n > kMaxGaussians) return fail(DGS_ERR_INVALID_ARG, "n = %d outside 0..2^28-1", s->n);
  if (s->rank < 0 || s->rank > 4) return fail(DGS_ERR_INVALID_ARG, "rank %d outside 0..4", s->rank);
  if (s->sh_degree != 0 && s->sh_degree != 1)
    return fail(DGS_ERR_INVALID_ARG, "sh_degree %d not 0 or 1", s->sh_degree);
  if (s->num_clusters < 1 || s->num_contexts < 1 ||
      (int64_t)s->num_clusters * s->num_contexts > 16384)
    return fail(DGS_ERR_INVALID_ARG, "packets C*K = %d*%d outside 1..16384", s->num_clusters,
                s->num_contexts);
  if (s->n > 0) {
    if (!s->mean || !s->log_scale || !s->quat || !s->opacity_logit || !s->color || !s->packet_layer)
      return fail(DGS_ERR_INVALID_ARG, "scene array pointer is NULL");
    if (s->rank > 0 && !s->temporal) return fail(DGS_ERR_INVALID_ARG, "temporal is NULL with rank > 0");
  }
  if (s->refine && (int64_t)s->n * 4 > kMaxGaussians)
    return fail(DGS_ERR_INVALID_ARG, "n = %d with refinement levels: 4n outside 0..2^28-1", s->n);
  return DGS_OK;
}

int check_states(const dgs_states *st, int P, int need_codes) {
  if (!st) return fail(DGS_ERR_INVALID_ARG, "states is NULL");
  if (st->num_states < 0) return fail(DGS_ERR_INVALID_ARG, "num_states %d < 0", st->num_states);
  if (need_codes && st->num_states > 0 && !st->codes) return fail(DGS_ERR_INVALID_ARG, "codes is NULL");
  for (int k = 0; k < 4; ++k)
    if (!isfinite(st->basis[k])) return fail(DGS_ERR_INVALID_ARG, "basis not finite");
  (void)P;
  return DGS_OK;
}

SceneArgs scene_args(const dgs_scene *s, const dgs_states *st) {
  SceneArgs a{};
  a.n = s->n;
  a.rank = s->rank;
  a.sh_degree = s->sh_degree;
  a.num_contexts = s->num_contexts;
  a.num_packets = s->num_clusters * s->num_contexts;
  a.mean = s->mean;
  a.log_scale = s->log_scale;
  a.quat = s->quat;
  a.opacity_logit = s->opacity_logit;
  a.color = s->color;
  a.temporal = s->temporal;
  a.packet_layer = s->packet_layer;
  a.affine = s->cluster_affine;
  a.refine = s->refine;
  a.refine_rows = s->refine ? 11 + (s->sh_degree == 0 ? 3 : 12) : 0;
  for (int k = 0; k < 4; ++k) a.basis[k] = (k < s->rank) ? st->basis[k] : 0.0f;
  return a;
}

CamArgs cam_args(const dgs_camera *c) {
  CamArgs a{};
  memcpy(a.R, c->R_cw, sizeof(a.R));
  memcpy(a.t, c->t_cw, sizeof(a.t));
  a.fx = c->fx; a.fy = c->fy; a.cx = c->cx; a.cy = c->cy; a.near_z = c->near_z;
  a.width = c->width; a.height = c->height;
  for (int k = 0; k < 3; ++k)
    a.campos[k] = (float)(-((double)c->R_cw[k] * c->t_cw[0] + (double)c->R_cw[3 + k] * c->t_cw[1] +
                            (double)c->R_cw[6 + k] * c->t_cw[2]));
  return a;
}

// Everything a call needs, validated.
struct Call {
  SceneArgs s;
  CamArgs c;
  TileArgs t;
  Tiling tiling;
  Layout L;
  int P;
  int records;  // projected records: n, or 4n (one per delivered depth) with refinement levels
};

int prepare(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
            const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, int need_codes, Call *call) {
  int rc;
  if ((rc = check_scene(scene)) || (rc = check_camera(cam))) return rc;
  const int P = scene->num_clusters * scene->num_contexts;
  if ((rc = check_states(states, P, need_codes))) return rc;
  if ((rc = check_tuning(cam, tun, &call->tiling))) return rc;
  if (cap < 0 || cap > (int64_t)0xFFFFFFFFll)
    return fail(DGS_ERR_INVALID_ARG, "instance capacity %lld outside 0..2^32-1", (long long)cap);
  if (!ws) return fail(DGS_ERR_INVALID_ARG, "workspace is NULL");
  if (((uintptr_t)ws) & 255u) return fail(DGS_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  call->P = P;
  call->records = scene->refine ? 4 * scene->n : scene->n;
  call->L = make_layout(call->records, P, call->tiling.tiles_x, call->tiling.tiles_y, states->num_states, cap);
  if (ws_bytes < call->L.total)
    return fail(DGS_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, call->L.total);
  call->s = scene_args(scene, states);
  call->c = cam_args(cam);
  call->t.tile_w = call->tiling.tw;
  call->t.tile_h = call->tiling.th;
  call->t.tiles_x = call->tiling.tiles_x;
  call->t.tiles_y = call->tiling.tiles_y;
  return DGS_OK;
}

// Header reset with the zeroing the binning needs (the tile difference array,
// and the (packet, layer) histogram when `plhist`), in one launch.
void clear_for_binning(const Call &cl, void *ws, int64_t cap, bool plhist, hipStream_t st) {
  const Layout &L = cl.L;
  launch_clear_header(at<Header>(ws, L.header), (unsigned long long)cap, st, at<uint32_t>(ws, L.tdiff),
                      (int64_t)(cl.tiling.tiles_x + 1) * (cl.tiling.tiles_y + 1),
                      plhist ? at<uint32_t>(ws, L.plhist) : nullptr, (int64_t)cl.P * kPlStride);
}

// Projection, depth sort, instance count and offsets, after clear_for_binning.
// `list_mode`: only the Gaussians listed in ws.list (count in
// header.n_active) take part.  `plhist`: the projection also counts every
// Gaussian per (packet, layer).  Returns whether the tile order was written
// as well (grids whose ranges come from the single-workgroup kernel).
bool project_and_count(const Call &cl, void *ws, bool list_mode, bool plhist, hipStream_t st) {
  const Layout &L = cl.L;
  Header *h = at<Header>(ws, L.header);
  const int n = cl.records;
  const uint32_t *list = list_mode ? at<uint32_t>(ws, L.present) : nullptr;
  const unsigned *nact = list_mode ? &h->n_active : nullptr;
  launch_geometry(cl.s, cl.c, cl.t, list, nact, n, at<float4>(ws, L.rec0), at<float4>(ws, L.rec1),
                  at<float4>(ws, L.rec2), at<uint2>(ws, L.rect), at<uint2>(ws, L.pbox), at<uint4>(ws, L.brec),
                  at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), st,
                  plhist && !list_mode ? at<uint32_t>(ws, L.plhist) : nullptr);
  // depth keys: 32 bits, 4 passes -> result back in dkey0/dval0
  launch_radix_sort(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), at<uint32_t>(ws, L.dkey1),
                    at<uint32_t>(ws, L.dval1), nact, 0, n, 0, 32, at<uint32_t>(ws, L.hist),
                    at<unsigned long long>(ws, L.part), st);
  if (super_path(cl.tiling.tiles_x, cl.tiling.tiles_y)) {
    // per-tile counts, ranges and the instance count straight from the rectangles
    return launch_tile_ranges(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), at<uint2>(ws, L.rect), nact, n,
                              cl.tiling.tiles_x, cl.tiling.tiles_y, h, at<uint32_t>(ws, L.tdiff),
                              at<uint32_t>(ws, L.tcnt), at<uint32_t>(ws, L.tstart),
                              at<unsigned long long>(ws, L.part), at<uint2>(ws, L.ranges), st,
                              /*tdiff_zeroed=*/true, at<uint32_t>(ws, L.tile_order));
  }
  launch_count(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), at<uint2>(ws, L.rect), nact, n,
               at<uint32_t>(ws, L.cnt), st);
  // offsets go to dkey1 (free after the depth sort)
  launch_scan_u32(at<uint32_t>(ws, L.cnt), at<uint32_t>(ws, L.dkey1), n, at<unsigned long long>(ws, L.part),
                  &h->instances, st);
  return false;
}

// Buffer holding the tile-sorted values after a binning.
const uint32_t *sorted_vals(const Call &cl, void *ws) {
  const int passes = (cl.tiling.tile_bits + 7) / 8;
  return (passes & 1) ? at<uint32_t>(ws, cl.L.tval1) : at<uint32_t>(ws, cl.L.tval0);
}

// Emission, tile sort and ranges; returns the sorted Gaussian ids.
const uint32_t *emit_and_sort(const Call &cl, void *ws, bool list_mode, int64_t cap, hipStream_t st) {
  const Layout &L = cl.L;
  Header *h = at<Header>(ws, L.header);
  const int n = cl.records;
  const unsigned *nact = list_mode ? &h->n_active : nullptr;
  if (super_path(cl.tiling.tiles_x, cl.tiling.tiles_y)) {
    // the ranges exist already (project_and_count); the two-level scatter puts every instance in place
    uint32_t *out = const_cast<uint32_t *>(sorted_vals(cl, ws));
    launch_super_scatter(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), at<uint2>(ws, L.rect), nact, n,
                         cl.tiling.tiles_x, cl.tiling.tiles_y, cl.t.tile_w, cl.t.tile_h, at<uint4>(ws, L.brec),
                         at<uint2>(ws, L.ranges), h, at<uint32_t>(ws, L.super_cnt),
                         at<uint32_t>(ws, L.super_tab), at<uint32_t>(ws, L.tkey0), at<uint32_t>(ws, L.tkey1), cap,
                         out, st);
    return out;
  }
  launch_emit(at<uint32_t>(ws, L.dval0), at<uint2>(ws, L.rect), at<uint32_t>(ws, L.dkey1),
              at<uint32_t>(ws, L.cnt), nact, n, cl.t.tiles_x, cl.t.tile_w, cl.t.tile_h, at<float4>(ws, L.rec0),
              at<float4>(ws, L.rec1), at<uint2>(ws, L.pbox), h, at<uint32_t>(ws, L.tkey0), at<uint32_t>(ws, L.tval0),
              st);
  // the last pass writes values only: tile ranges come from the rectangles
  const int r = launch_radix_sort(at<uint32_t>(ws, L.tkey0), at<uint32_t>(ws, L.tval0), at<uint32_t>(ws, L.tkey1),
                                  at<uint32_t>(ws, L.tval1), &h->instances, 1, cap, 0, cl.tiling.tile_bits,
                                  at<uint32_t>(ws, L.hist), at<unsigned long long>(ws, L.part), st,
                                  /*last_pass_keys=*/false);
  launch_tile_ranges(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), at<uint2>(ws, L.rect), nact, n,
                     cl.tiling.tiles_x, cl.tiling.tiles_y, h, at<uint32_t>(ws, L.tdiff), at<uint32_t>(ws, L.tcnt),
                     at<uint32_t>(ws, L.tstart), at<unsigned long long>(ws, L.part), at<uint2>(ws, L.ranges), st);
  return r ? at<uint32_t>(ws, L.tval1) : at<uint32_t>(ws, L.tval0);
}


// List entries per LDS batch (validated by check_tuning).
int lds_batch(const dgs_tuning *tun) { return (tun && tun->lds_batch) ? tun->lds_batch : 256; }

// 0 automatic, 1 persistent, 2 grid (validated by check_tuning)
int launch_kind(const dgs_tuning *tun) {
  if (!tun) return 0;
  return (tun->flags & DGS_TUNE_PERSISTENT) ? 1 : (tun->flags & DGS_TUNE_GRID) ? 2 : 0;
}

int group_size(const dgs_tuning *tun, int W, int max_s) {
  int S = (tun && tun->states_per_group) ? tun->states_per_group : 16;
  if (S < 1) S = 1;
  if (S > max_s) S = max_s;
  int p = 1;
  while (p < S) p <<= 1;
  if (p > S) p >>= 1;  // round down to a power of two
  S = p;
  int need = 1;
  while (need < W) need <<= 1;
  if (W > 0 && S > need) S = need;
  return S;
}

CompositeArgs composite_args(const Call &cl, void *ws, const uint32_t *vals, const dgs_states *states,
                             const uint32_t *visbits, int groups) {
  CompositeArgs a{};
  a.rec0 = at<float4>(ws, cl.L.rec0);
  a.rec1 = at<float4>(ws, cl.L.rec1);
  a.rec2 = at<float4>(ws, cl.L.rec2);
  a.vals = vals;
  a.ranges = at<uint2>(ws, cl.L.ranges);
  a.tile_order = at<uint32_t>(ws, cl.L.tile_order);
  a.visbits = visbits;
  a.P4 = cl.P * 4;
  a.num_states = states->num_states;
  a.width = cl.c.width;
  a.height = cl.c.height;
  a.tiles_x = cl.tiling.tiles_x;
  a.tiles_y = cl.tiling.tiles_y;
  a.groups = groups;
  for (int k = 0; k < 3; ++k) a.bg[k] = states->background[k];
  return a;
}

int device_cus() {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus > 0 ? cus : 256;
}

// Validation and argument set-up shared by dgs_utility_count and dgs_utility.
int utility_prepare(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *contexts,
                    const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, const int32_t *context_group,
                    const uint16_t *group_pl, int32_t num_groups, void *uws, size_t uws_bytes,
                    int64_t item_capacity, Call *cl, UtilArgs *u) {
  // the render workspace is read only in its state-independent sections
  if (!contexts) return fail(DGS_ERR_INVALID_ARG, "contexts is NULL");
  dgs_states none = *contexts;
  none.num_states = 0;
  int rc = prepare(scene, cam, &none, tun, ws, ws_bytes, cap, 0, cl);
  if (rc) return rc;
  if ((rc = check_states(contexts, cl->P, 1))) return rc;
  if (num_groups < 1 || num_groups > 1 << 20) return fail(DGS_ERR_INVALID_ARG, "num_groups %d outside 1..2^20", num_groups);
  if (!group_pl) return fail(DGS_ERR_INVALID_ARG, "group_pl is NULL");
  if (contexts->num_states > 0 && !context_group) return fail(DGS_ERR_INVALID_ARG, "context_group is NULL");
  if (contexts->num_states > (1 << 24)) return fail(DGS_ERR_INVALID_ARG, "more than 2^24 contexts");
  if (item_capacity < 0 || item_capacity > (int64_t)0x7FFFFFFFll)
    return fail(DGS_ERR_INVALID_ARG, "item capacity %lld outside 0..2^31-1", (long long)item_capacity);
  if (!uws) return fail(DGS_ERR_INVALID_ARG, "utility workspace is NULL");
  if (((uintptr_t)uws) & 255u) return fail(DGS_ERR_INVALID_ARG, "utility workspace not 256-byte aligned");
  const UtilLayout U = make_util_layout(cl->P, cl->tiling.tiles, num_groups, contexts->num_states, item_capacity);
  if (uws_bytes < U.total)
    return fail(DGS_ERR_WORKSPACE, "utility workspace %zu bytes < %zu needed", uws_bytes, U.total);
  *u = UtilArgs{};
  u->hdr = at<UtilHeader>(uws, U.hdr);
  u->pl2g = at<int>(uws, U.pl2g);
  u->core = at<uint32_t>(uws, U.core);
  u->region = at<uint32_t>(uws, U.region);
  u->wcount = at<uint32_t>(uws, U.wcount);
  u->wprefix = at<uint32_t>(uws, U.wprefix);
  u->region_tiles = at<uint32_t>(uws, U.region_tiles);
  u->group_base = at<uint32_t>(uws, U.group_base);
  u->icount = at<uint32_t>(uws, U.icount);
  u->item_base = at<uint32_t>(uws, U.item_base);
  u->bcount = at<uint32_t>(uws, U.bcount);
  u->bbase = at<uint32_t>(uws, U.bbase);
  u->bad = at<uint32_t>(uws, U.bad);
  u->pvis = at<uint32_t>(uws, U.pvis);
  u->parts = at<unsigned long long>(uws, U.parts);
  u->partial = at<float>(uws, U.partial);
  u->patches = at<float>(uws, U.patches);
  u->item_total = &u->hdr->items;
  u->queue = u->hdr->queue;
  u->item_capacity = (uint64_t)item_capacity;
  u->num_contexts = contexts->num_states;
  u->refined = scene->refine != nullptr;
  u->words = (int)U.words;
  u->tiles_x = cl->tiling.tiles_x;
  u->tiles_y = cl->tiling.tiles_y;
  u->width = cl->c.width;
  u->height = cl->c.height;
  u->context_group = context_group;
  return DGS_OK;
}

// Group tables, regions and per-context work items (from the last dgs_bin).
void utility_setup(const Call &cl, void *ws, const UtilArgs &u, const dgs_states *contexts, const uint16_t *group_pl,
                   int G, hipStream_t st) {
  launch_clear_util_header(u.hdr, st);
  const int rx = (10 + cl.tiling.tw - 1) / cl.tiling.tw, ry = (10 + cl.tiling.th - 1) / cl.tiling.th;
  launch_group_setup(u, group_pl, G, cl.P, at<float4>(ws, cl.L.rec0), at<uint2>(ws, cl.L.rect), cl.records, rx, ry,
                     st);
  if (u.num_contexts > 0) launch_pair_setup(u, contexts->codes, group_pl, G, cl.P, st);
}

int utility_status(const UtilHeader &h, int64_t item_capacity) {
  if (h.bad_group & 1u) return fail(DGS_ERR_INVALID_ARG, "a group names a packet outside the scene");
  if (h.bad_group & 2u) return fail(DGS_ERR_INVALID_ARG, "two groups name the same (packet, layer)");
  if (h.bad_context)
    return fail(DGS_ERR_INVALID_ARG, "a context does not hold its group's packet at exactly the group's layer");
  if ((int64_t)h.items > item_capacity)
    return fail(DGS_ERR_OVERFLOW, "%llu work items exceed capacity %lld", h.items, (long long)item_capacity);
  return DGS_OK;
}

}  // namespace

extern "C" {

int dgs_abi_version(void) { return DGS_ABI_VERSION; }

const char *dgs_status_string(int status) {
  switch (status) {
    case DGS_OK: return "ok";
    case DGS_ERR_INVALID_ARG: return "invalid argument";
    case DGS_ERR_WORKSPACE: return "workspace too small";
    case DGS_ERR_OVERFLOW: return "instance capacity exceeded";
    case DGS_ERR_HIP: return "HIP runtime error";
    case DGS_ERR_UNSUPPORTED: return "unsupported tuning";
    default: return "unknown status";
  }
}

const char *dgs_last_error(void) { return g_err.c_str(); }

size_t dgs_workspace_bytes(int32_t n, int32_t num_packets, const dgs_camera *cam, const dgs_tuning *tun,
                           int32_t max_states, int64_t instance_capacity) {
  Tiling t;
  if (n < 0 || n > kMaxGaussians || num_packets < 1 || num_packets > 16384 || max_states < 0 ||
      instance_capacity < 0 || instance_capacity > (int64_t)0xFFFFFFFFll)
    return 0;
  if (check_camera(cam) || check_tuning(cam, tun, &t)) return 0;
  return make_layout(n, num_packets, t.tiles_x, t.tiles_y, max_states, instance_capacity).total;
}

int dgs_count_instances(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                        const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t *instances, void *stream) {
  g_err.clear();
  if (!instances) return fail(DGS_ERR_INVALID_ARG, "instances is NULL");
  if (!states) return fail(DGS_ERR_INVALID_ARG, "states is NULL");
  dgs_states st0 = *states;
  st0.num_states = 0;  // no per-state buffers needed
  Call cl;
  int rc = prepare(scene, cam, &st0, tun, ws, ws_bytes, 0, 0, &cl);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = refuse_capture(st, "dgs_count_instances"))) return rc;
  Header *h = at<Header>(ws, cl.L.header);
  clear_for_binning(cl, ws, 0, false, st);
  project_and_count(cl, ws, false, false, st);
  if ((rc = hip_check("count_instances launch"))) return rc;
  Header hh;
  if (hipMemcpyAsync(&hh, h, sizeof(Header), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return hip_check("count_instances copy");
  *instances = (int64_t)hh.instances;
  return DGS_OK;
}

int dgs_bin(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states, const dgs_tuning *tun,
            void *ws, size_t ws_bytes, int64_t cap, void *stream) {
  g_err.clear();
  Call cl;
  int rc = prepare(scene, cam, states, tun, ws, ws_bytes, cap, 0, &cl);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  clear_for_binning(cl, ws, cap, true, st);
  const bool ordered = project_and_count(cl, ws, false, true, st);  // also counts the (packet, layer) histogram
  emit_and_sort(cl, ws, false, cap, st);
  if (!ordered) launch_tile_order(at<uint2>(ws, cl.L.ranges), cl.tiling.tiles, at<uint32_t>(ws, cl.L.tile_order), st);
  return hip_check("bin launch");
}

namespace {

// Masked compositing of every state from the lists of the last dgs_bin.
// mode 0: images, 1: PSNR partials + finalisation, 2: work counters.
int composite_call(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                   const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, int mode, float *image,
                   float *tfinal, const float *reference, float *psnr, unsigned long long *counters,
                   void *stream) {
  Call cl;
  int rc = prepare(scene, cam, states, tun, ws, ws_bytes, cap, 1, &cl);
  if (rc) return rc;
  const int W = states->num_states;
  if (mode == 0 && W > 0 && !image) return fail(DGS_ERR_INVALID_ARG, "image is NULL");
  if (mode == 1 && W > 0 && (!reference || !psnr)) return fail(DGS_ERR_INVALID_ARG, "reference / psnr is NULL");
  if (mode == 2 && !counters) return fail(DGS_ERR_INVALID_ARG, "counters is NULL");
  hipStream_t st = (hipStream_t)stream;
  if (mode == 2) launch_fill_u64(counters, 4, st);
  if (W == 0) return hip_check("composite launch");
  const int S = group_size(tun, W, 32);
  const int groups = (W + S - 1) / S;
  uint32_t *visbits = at<uint32_t>(ws, cl.L.visbits);
  uint32_t *order = at<uint32_t>(ws, cl.L.state_order);
  launch_state_order(states->codes, at<uint32_t>(ws, cl.L.plhist), W, cl.P, at<uint32_t>(ws, cl.L.state_cnt),
                     order, st);
  launch_visbits(states->codes, order, W, cl.P, S, scene->refine != nullptr, visbits, st);
  CompositeArgs a = composite_args(cl, ws, sorted_vals(cl, ws), states, visbits, groups);
  a.state_order = order;
  a.launch_states = W;
  a.image = image;
  a.tfinal = tfinal;
  a.reference = reference;
  a.psnr_part = at<float>(ws, cl.L.psnr_part);
  a.counters = counters;
  a.queues = at<unsigned int>(ws, cl.L.queues);
  if (launch_composite(a, S, cl.tiling.tw, cl.tiling.th, mode, launch_kind(tun), lds_batch(tun), st))
    return fail(DGS_ERR_UNSUPPORTED, "no composite variant for S=%d", S);
  if (mode == 1)
    launch_psnr_finalize(a.psnr_part, W, cl.tiling.tiles, (int64_t)cl.c.width * cl.c.height, psnr, st);
  return hip_check("composite launch");
}

}  // namespace

int dgs_composite(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                  const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, float *image, float *tfinal,
                  void *stream) {
  g_err.clear();
  return composite_call(scene, cam, states, tun, ws, ws_bytes, cap, 0, image, tfinal, nullptr, nullptr, nullptr,
                        stream);
}

int dgs_composite_psnr(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                       const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, const float *reference,
                       float *psnr, void *stream) {
  g_err.clear();
  return composite_call(scene, cam, states, tun, ws, ws_bytes, cap, 1, nullptr, nullptr, reference, psnr, nullptr,
                        stream);
}

int dgs_composite_stats(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                        const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap,
                        unsigned long long *counters, void *stream) {
  g_err.clear();
  return composite_call(scene, cam, states, tun, ws, ws_bytes, cap, 2, nullptr, nullptr, nullptr, nullptr,
                        counters, stream);
}

int dgs_render(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states, const dgs_tuning *tun,
               void *ws, size_t ws_bytes, int64_t cap, float *image, float *tfinal, void *stream) {
  g_err.clear();
  Call cl;
  int rc = prepare(scene, cam, states, tun, ws, ws_bytes, cap, 1, &cl);
  if (rc) return rc;
  if (states->num_states > 0 && !image) return fail(DGS_ERR_INVALID_ARG, "image is NULL");
  if (states->num_states == 0) return DGS_OK;
  if ((rc = dgs_bin(scene, cam, states, tun, ws, ws_bytes, cap, stream))) return rc;
  return dgs_composite(scene, cam, states, tun, ws, ws_bytes, cap, image, tfinal, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free render.  The workspace of dgs_render_noalloc is a static
// device array of fixed size (every GPU the library runs on holds its own
// copy until the process ends).  In host code `scratch` only names the
// symbol: its device address comes from hipGetSymbolAddress, looked up once
// per device on that device's first call and kept in noalloc_ptr.
constexpr size_t kNoAllocScratchBytes = DGS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
void *noalloc_ptr[kMaxDevices];

// Device address of the current device's scratch (looked up on first use).
int noalloc_scratch(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(DGS_ERR_HIP, "dgs_render_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  }
  if (dev < 0 || dev >= kMaxDevices)
    return fail(DGS_ERR_UNSUPPORTED, "dgs_render_noalloc: device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(DGS_ERR_HIP, "dgs_render_noalloc: address of the static scratch on device %d: %s", dev,
                  hipGetErrorString(e));
    }
    noalloc_ptr[dev] = p;
  }
  *out = noalloc_ptr[dev];
  return DGS_OK;
}

__global__ void k_report_instances(const Header *h, int64_t *out) { *out = (int64_t)h->instances; }

}  // namespace

extern "C" {

int dgs_render_noalloc(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                       const dgs_tuning *tun, int64_t cap, float *image, float *tfinal, int64_t *instances,
                       void *stream) {
  g_err.clear();
  // sizes first, on the host: nothing reaches the device for a call that does not fit
  int rc;
  if ((rc = check_scene(scene)) || (rc = check_camera(cam))) return rc;
  const int P = scene->num_clusters * scene->num_contexts;
  if ((rc = check_states(states, P, 1))) return rc;
  Tiling t;
  if ((rc = check_tuning(cam, tun, &t))) return rc;
  if (cap < 0 || cap > (int64_t)0xFFFFFFFFll)
    return fail(DGS_ERR_INVALID_ARG, "instance capacity %lld outside 0..2^32-1", (long long)cap);
  const int records = scene->refine ? 4 * scene->n : scene->n;
  const size_t need = make_layout(records, P, t.tiles_x, t.tiles_y, states->num_states, cap).total;
  if (need > kNoAllocScratchBytes)
    return fail(DGS_ERR_WORKSPACE,
                "dgs_render_noalloc: this call needs %zu bytes of workspace, the static scratch holds %zu "
                "(use fewer Gaussians, states, tiles or a smaller instance capacity, or dgs_render)",
                need, kNoAllocScratchBytes);
  if (states->num_states > 0 && !image) return fail(DGS_ERR_INVALID_ARG, "image is NULL");
  if (states->num_states == 0 && !instances) return DGS_OK;
  void *ws = nullptr;
  if ((rc = noalloc_scratch(&ws))) return rc;
  if ((rc = dgs_bin(scene, cam, states, tun, ws, kNoAllocScratchBytes, cap, stream))) return rc;
  if (states->num_states > 0 &&
      (rc = dgs_composite(scene, cam, states, tun, ws, kNoAllocScratchBytes, cap, image, tfinal, stream)))
    return rc;
  if (instances) {
    Call cl;
    if ((rc = prepare(scene, cam, states, tun, ws, kNoAllocScratchBytes, cap, 1, &cl))) return rc;
    k_report_instances<<<1, 1, 0, (hipStream_t)stream>>>(at<Header>(ws, cl.L.header), instances);
  }
  return hip_check("render_noalloc launch");
}

int dgs_render_per_state(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                         const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, float *image,
                         float *tfinal, void *stream) {
  g_err.clear();
  Call cl;
  int rc = prepare(scene, cam, states, tun, ws, ws_bytes, cap, 1, &cl);
  if (rc) return rc;
  if (states->num_states > 0 && !image) return fail(DGS_ERR_INVALID_ARG, "image is NULL");
  hipStream_t st = (hipStream_t)stream;
  const int W = states->num_states;
  const int n = cl.s.n;
  Header *h = at<Header>(ws, cl.L.header);
  for (int w = 0; w < W; ++w) {
    clear_for_binning(cl, ws, cap, false, st);
    // compaction of the delivered Gaussians (flags -> scan -> scatter)
    launch_present_flags(states->codes + (int64_t)w * cl.P, scene->packet_layer, n, cl.P,
                         at<uint32_t>(ws, cl.L.cnt), st);
    launch_scan_u32(at<uint32_t>(ws, cl.L.cnt), at<uint32_t>(ws, cl.L.dkey1), n,
                    at<unsigned long long>(ws, cl.L.part), &h->instances, st);
    launch_present_scatter(at<uint32_t>(ws, cl.L.cnt), at<uint32_t>(ws, cl.L.dkey1), n,
                           states->codes + (int64_t)w * cl.P, scene->packet_layer, scene->refine != nullptr,
                           at<uint32_t>(ws, cl.L.present), &h->instances, h, st);
    const bool ordered = project_and_count(cl, ws, true, false, st);
    const uint32_t *vals = emit_and_sort(cl, ws, true, cap, st);
    if (!ordered)
      launch_tile_order(at<uint2>(ws, cl.L.ranges), cl.tiling.tiles, at<uint32_t>(ws, cl.L.tile_order), st);
    CompositeArgs a = composite_args(cl, ws, vals, states, nullptr, 1);
    a.image = image;
    a.tfinal = tfinal;
    a.state_offset = w;
    a.launch_states = 1;
    if (launch_composite(a, 1, cl.tiling.tw, cl.tiling.th, 0, 2, 256, st))
      return fail(DGS_ERR_UNSUPPORTED, "no composite variant for S=1");
  }
  return hip_check("render_per_state launch");
}

int dgs_render_psnr(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states,
                    const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, const float *reference,
                    float *psnr, void *stream) {
  g_err.clear();
  Call cl;
  int rc = prepare(scene, cam, states, tun, ws, ws_bytes, cap, 1, &cl);
  if (rc) return rc;
  const int W = states->num_states;
  if (W > 0 && (!reference || !psnr)) return fail(DGS_ERR_INVALID_ARG, "reference / psnr is NULL");
  if (W == 0) return DGS_OK;
  if ((rc = dgs_bin(scene, cam, states, tun, ws, ws_bytes, cap, stream))) return rc;
  return dgs_composite_psnr(scene, cam, states, tun, ws, ws_bytes, cap, reference, psnr, stream);
}

int dgs_backward(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *states, const dgs_tuning *tun,
                 void *ws, size_t ws_bytes, int64_t cap, const float *image, const float *grad_image,
                 const dgs_scene_grad *grad, void *stream) {
  g_err.clear();
  Call cl;
  int rc = prepare(scene, cam, states, tun, ws, ws_bytes, cap, 1, &cl);
  if (rc) return rc;
  if (!grad || (scene->n > 0 && (!grad->mean || !grad->log_scale || !grad->quat || !grad->opacity_logit ||
                                 !grad->color || (scene->rank > 0 && !grad->temporal) ||
                                 (scene->refine && !grad->refine))))
    return fail(DGS_ERR_INVALID_ARG, "gradient pointer is NULL");
  const int W = states->num_states;
  if (W > 0 && (!image || !grad_image)) return fail(DGS_ERR_INVALID_ARG, "image / grad_image is NULL");
  hipStream_t st = (hipStream_t)stream;
  const int n = cl.records;  // 2D gradients per projected record
  float *g2d = at<float>(ws, cl.L.grad2d);
  launch_fill_f32(g2d, (int64_t)9 * n, 0.0f, st);
  if (W > 0) {
    const int S = group_size(tun, W, 8);
    const int groups = (W + S - 1) / S;
    uint32_t *visbits = at<uint32_t>(ws, cl.L.visbits);
    uint32_t *order = at<uint32_t>(ws, cl.L.state_order);
    launch_state_order(states->codes, at<uint32_t>(ws, cl.L.plhist), W, cl.P, at<uint32_t>(ws, cl.L.state_cnt),
                       order, st);
    launch_visbits(states->codes, order, W, cl.P, S, scene->refine != nullptr, visbits, st);
    CompositeBwdArgs b{};
    b.tile_order = at<uint32_t>(ws, cl.L.tile_order);
    b.state_order = order;
    b.rec0 = at<float4>(ws, cl.L.rec0);
    b.rec1 = at<float4>(ws, cl.L.rec1);
    b.rec2 = at<float4>(ws, cl.L.rec2);
    b.vals = sorted_vals(cl, ws);
    b.ranges = at<uint2>(ws, cl.L.ranges);
    b.visbits = visbits;
    b.P4 = cl.P * 4;
    b.num_states = W;
    b.width = cl.c.width;
    b.height = cl.c.height;
    b.tiles_x = cl.tiling.tiles_x;
    b.tiles_y = cl.tiling.tiles_y;
    b.groups = groups;
    b.image = image;
    b.grad_image = grad_image;
    b.g2d = g2d;
    b.n = n;
    if (launch_composite_bwd(b, S, cl.tiling.tw, cl.tiling.th, st))
      return fail(DGS_ERR_UNSUPPORTED, "no backward variant for S=%d", S);
  }
  launch_geometry_bwd(cl.s, cl.c, g2d, grad->mean, grad->log_scale, grad->quat, grad->opacity_logit,
                      grad->color, grad->temporal, grad->refine, st);
  return hip_check("backward launch");
}

int dgs_workspace_sections(int32_t n, int32_t num_packets, const dgs_camera *cam, const dgs_tuning *tun,
                           int32_t max_states, int64_t instance_capacity, dgs_workspace_view *out) {
  g_err.clear();
  Tiling t;
  int rc;
  if (!out) return fail(DGS_ERR_INVALID_ARG, "out is NULL");
  if (n < 0 || num_packets < 1 || num_packets > 16384 || max_states < 0 || instance_capacity < 0 ||
      instance_capacity > (int64_t)0xFFFFFFFFll)
    return fail(DGS_ERR_INVALID_ARG, "sizes out of range");
  if ((rc = check_camera(cam)) || (rc = check_tuning(cam, tun, &t))) return rc;
  const Layout L = make_layout(n, num_packets, t.tiles_x, t.tiles_y, max_states, instance_capacity);
  const int passes = (t.tile_bits + 7) / 8;
  out->rec0 = L.rec0;
  out->rec1 = L.rec1;
  out->rec2 = L.rec2;
  out->rect = L.rect;
  out->ranges = L.ranges;
  out->sorted_ids = (passes & 1) ? L.tval1 : L.tval0;
  out->tiles_x = t.tiles_x;
  out->tiles_y = t.tiles_y;
  return DGS_OK;
}

int dgs_composite_launch(const dgs_camera *cam, const dgs_tuning *tun, int32_t num_states, int32_t *states_per_group,
                         int32_t *persistent, int64_t *workgroups, int64_t *work_items, int32_t *lds_batch_out) {
  g_err.clear();
  Tiling t;
  int rc;
  if (!states_per_group || !persistent || !workgroups || !work_items || !lds_batch_out)
    return fail(DGS_ERR_INVALID_ARG, "output pointer is NULL");
  if (num_states < 0) return fail(DGS_ERR_INVALID_ARG, "num_states < 0");
  if ((rc = check_camera(cam)) || (rc = check_tuning(cam, tun, &t))) return rc;
  const int S = group_size(tun, num_states, 32);
  CompositePlan p;
  if (plan_composite(S, t.tw, t.th, t.tiles, (num_states + S - 1) / S, launch_kind(tun), lds_batch(tun), &p))
    return fail(DGS_ERR_UNSUPPORTED, "no composite variant for S=%d", S);
  *states_per_group = S;
  *persistent = p.persistent ? 1 : 0;
  *workgroups = p.workgroups;
  *work_items = p.items;
  *lds_batch_out = p.lds_batch;
  return hip_check("occupancy query");
}

int dgs_check(void *ws, size_t ws_bytes, int64_t *instances, void *stream) {
  g_err.clear();
  if (!ws || ws_bytes < sizeof(Header)) return fail(DGS_ERR_INVALID_ARG, "workspace missing");
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = refuse_capture(st, "dgs_check"))) return rc;
  Header hh;
  if (hipMemcpyAsync(&hh, ws, sizeof(Header), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return hip_check("check copy");
  if (instances) *instances = (int64_t)hh.instances;
  if (hh.overflow)
    return fail(DGS_ERR_OVERFLOW, "%llu instances exceed capacity %llu", hh.instances, hh.capacity);
  return hip_check("check");
}

size_t dgs_utility_workspace_bytes(int32_t num_packets, const dgs_camera *cam, const dgs_tuning *tun,
                                   int32_t num_groups, int32_t num_contexts, int64_t item_capacity) {
  g_err.clear();
  Tiling t;
  if (num_packets < 1 || num_packets > 16384 || num_groups < 1 || num_groups > 1 << 20 || num_contexts < 0 ||
      num_contexts > (1 << 24) || item_capacity < 0 || item_capacity > (int64_t)0x7FFFFFFFll)
    return 0;
  if (check_camera(cam) || check_tuning(cam, tun, &t)) return 0;
  return make_util_layout(num_packets, t.tiles, num_groups, num_contexts, item_capacity).total;
}

int dgs_utility_count(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *contexts,
                      const dgs_tuning *tun, void *ws, size_t ws_bytes, int64_t cap, const int32_t *context_group,
                      const uint16_t *group_pl, int32_t num_groups, void *uws, size_t uws_bytes, int64_t *items,
                      void *stream) {
  g_err.clear();
  if (!items) return fail(DGS_ERR_INVALID_ARG, "items is NULL");
  Call cl;
  UtilArgs u;
  int rc = utility_prepare(scene, cam, contexts, tun, ws, ws_bytes, cap, context_group, group_pl, num_groups, uws,
                           uws_bytes, 0, &cl, &u);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = refuse_capture(st, "dgs_utility_count"))) return rc;
  utility_setup(cl, ws, u, contexts, group_pl, num_groups, st);
  UtilHeader h;
  if (hipMemcpyAsync(&h, u.hdr, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return hip_check("utility count");
  *items = (int64_t)h.items;
  if ((rc = utility_status(h, INT64_MAX))) return rc;
  return hip_check("utility count");
}

int dgs_utility(const dgs_scene *scene, const dgs_camera *cam, const dgs_states *contexts, const dgs_tuning *tun,
                void *ws, size_t ws_bytes, int64_t cap, const int32_t *context_group, const uint16_t *group_pl,
                int32_t num_groups, const float *reference, float lambda, void *uws, size_t uws_bytes,
                int64_t item_capacity, float *delta, void *stream) {
  g_err.clear();
  Call cl;
  UtilArgs u;
  int rc = utility_prepare(scene, cam, contexts, tun, ws, ws_bytes, cap, context_group, group_pl, num_groups, uws,
                           uws_bytes, item_capacity, &cl, &u);
  if (rc) return rc;
  if (contexts->num_states > 0 && (!reference || !delta))
    return fail(DGS_ERR_INVALID_ARG, "reference / delta is NULL");
  if (!isfinite(lambda)) return fail(DGS_ERR_INVALID_ARG, "lambda not finite");
  if (contexts->num_states == 0) return DGS_OK;
  hipStream_t st = (hipStream_t)stream;
  u.reference = reference;
  u.lambda = lambda;
  u.delta = delta;
  utility_setup(cl, ws, u, contexts, group_pl, num_groups, st);
  CompositeArgs a = composite_args(cl, ws, sorted_vals(cl, ws), contexts, u.pvis, 1);
  a.image = u.patches;
  a.queues = u.queue;
  a.pair.item_total = u.item_total;
  a.pair.item_capacity = u.item_capacity;
  a.pair.num_contexts = u.num_contexts;
  a.pair.item_base = u.item_base;
  a.pair.context_group = context_group;
  a.pair.group_base = u.group_base;
  a.pair.region_tiles = u.region_tiles;
  a.pair.bundle_total = &u.hdr->bundle_items;
  a.pair.bundle_base = u.bbase;
  a.pair.bad = u.bad;
  const int cus = device_cus();
  if (launch_composite_pairs(a, cl.tiling.tw, cl.tiling.th, cus * 8, st))
    return fail(DGS_ERR_UNSUPPORTED, "no pair compositing variant for this tile shape");
  if (launch_pair_ssim(u, cl.tiling.tw, cl.tiling.th, cus * 4, st))
    return fail(DGS_ERR_UNSUPPORTED, "no pair SSIM variant for this tile shape");
  return hip_check("utility launch");
}

int dgs_utility_check(void *uws, size_t uws_bytes, int64_t item_capacity, int64_t *items, void *stream) {
  g_err.clear();
  if (!uws || uws_bytes < sizeof(UtilHeader)) return fail(DGS_ERR_INVALID_ARG, "utility workspace missing");
  hipStream_t st = (hipStream_t)stream;
  int rc0;
  if ((rc0 = refuse_capture(st, "dgs_utility_check"))) return rc0;
  UtilHeader h;
  if (hipMemcpyAsync(&h, uws, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return hip_check("utility check copy");
  if (items) *items = (int64_t)h.items;
  int rc = utility_status(h, item_capacity);
  if (rc) return rc;
  return hip_check("utility check");
}

size_t dgs_distortion_scratch_bytes(int32_t num_images, int32_t width, int32_t height) {
  if (num_images < 0 || width < 1 || height < 1 || width > 16384 || height > 16384) return 0;
  return (size_t)num_images * (size_t)ceil_div(width, 16) * (size_t)ceil_div(height, 16) * 2 * sizeof(double) + 8;
}

int dgs_distortion(const float *images, int32_t num_images, int32_t width, int32_t height, const float *reference,
                   float lambda, void *scratch, size_t scratch_bytes, float *d, void *stream) {
  g_err.clear();
  if (num_images < 0 || width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(DGS_ERR_INVALID_ARG, "sizes out of range");
  if (num_images == 0) return DGS_OK;
  if (!images || !reference || !d || !scratch) return fail(DGS_ERR_INVALID_ARG, "pointer is NULL");
  if (((uintptr_t)scratch) & 7u) return fail(DGS_ERR_INVALID_ARG, "scratch not 8-byte aligned");
  if (!isfinite(lambda)) return fail(DGS_ERR_INVALID_ARG, "lambda not finite");
  if (scratch_bytes < dgs_distortion_scratch_bytes(num_images, width, height))
    return fail(DGS_ERR_WORKSPACE, "scratch %zu bytes < %zu needed", scratch_bytes,
                dgs_distortion_scratch_bytes(num_images, width, height));
  if (num_images > 65535) return fail(DGS_ERR_INVALID_ARG, "more than 65535 images per call");
  launch_distortion(images, num_images, width, height, reference, lambda, (double *)scratch, d, (hipStream_t)stream);
  return hip_check("distortion launch");
}

int dgs_risk_adjusted(const float *values, const int32_t *offsets, int32_t num_groups, float alpha, float beta,
                      float quantile, float *out, void *stream) {
  g_err.clear();
  if (num_groups < 0) return fail(DGS_ERR_INVALID_ARG, "num_groups < 0");
  if (num_groups == 0) return DGS_OK;
  if (!values || !offsets || !out) return fail(DGS_ERR_INVALID_ARG, "pointer is NULL");
  if (!isfinite(alpha) || !isfinite(beta) || !(quantile >= 0.0f && quantile <= 1.0f))
    return fail(DGS_ERR_INVALID_ARG, "alpha / beta not finite or quantile outside [0, 1]");
  launch_risk_adjusted(values, offsets, num_groups, alpha, beta, quantile, out, (hipStream_t)stream);
  return hip_check("risk launch");
}

int dgs_sample_states(const dgs_channel *channels, int32_t num_states, int32_t num_packets, int32_t num_layers,
                      uint64_t seed, uint8_t *codes, void *stream) {
  g_err.clear();
  static_assert(sizeof(dgs_channel) == sizeof(SamplerChannel), "dgs_channel layout");
  if (num_states < 0) return fail(DGS_ERR_INVALID_ARG, "num_states < 0");
  if (num_packets < 1 || num_packets > 16384) return fail(DGS_ERR_INVALID_ARG, "num_packets %d outside 1..16384", num_packets);
  if (num_layers < 1 || num_layers > 4) return fail(DGS_ERR_INVALID_ARG, "num_layers %d outside 1..4", num_layers);
  if (num_states == 0) return DGS_OK;
  if (!channels || !codes) return fail(DGS_ERR_INVALID_ARG, "channels / codes is NULL");
  launch_sample_states(reinterpret_cast<const SamplerChannel *>(channels), num_states, num_packets, num_layers, seed,
                       codes, (hipStream_t)stream);
  return hip_check("sample_states launch");
}

// ---------------------------------------------------------------- objective
static bool finite_weight(float v) { return isfinite(v) && v >= 0.0f; }

size_t dgs_objective_scratch_bytes(int32_t num_images, int32_t width, int32_t height, int32_t num_temporal) {
  if (num_images < 0 || num_images > kObjMaxImages || width < 1 || height < 1 || width > 16384 ||
      height > 16384 || num_temporal < 0 || num_temporal > kObjMaxPairs)
    return 0;
  return make_obj_layout(num_images, width, height, num_temporal).total;
}

int dgs_objective(const float *images, int32_t num_images, int32_t width, int32_t height, const float *targets,
                  int32_t num_targets, const int32_t *target_of, const int32_t *expect, int32_t num_expect,
                  const int32_t *anchor, int32_t num_anchor, const int32_t *mono, int32_t num_mono,
                  const int32_t *temporal, int32_t num_temporal, const dgs_objective_weights *w, float *loss,
                  float *distortion, float *grad, void *scratch, size_t scratch_bytes, void *stream) {
  g_err.clear();
  if (num_images < 0 || num_images > kObjMaxImages)
    return fail(DGS_ERR_INVALID_ARG, "num_images %d outside 0..%d", num_images, kObjMaxImages);
  if (width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(DGS_ERR_INVALID_ARG, "image size %dx%d outside 1..16384", width, height);
  if (num_expect < 0 || num_expect > kObjMaxExpect)
    return fail(DGS_ERR_INVALID_ARG, "num_expect %d outside 0..%d", num_expect, kObjMaxExpect);
  if (num_anchor < 0 || num_anchor > kObjMaxPairs || num_mono < 0 || num_mono > kObjMaxPairs ||
      num_temporal < 0 || num_temporal > kObjMaxPairs)
    return fail(DGS_ERR_INVALID_ARG, "anchor / pair counts outside 0..%d", kObjMaxPairs);
  if (!w) return fail(DGS_ERR_INVALID_ARG, "weights is NULL");
  if (!finite_weight(w->lambda_ssim) || !finite_weight(w->lambda_c) || !finite_weight(w->lambda_t) ||
      !finite_weight(w->lambda_m) || !finite_weight(w->lambda_a))
    return fail(DGS_ERR_INVALID_ARG, "weights must be finite and >= 0");
  if (!(w->alpha > 0.0f && w->alpha <= 1.0f)) return fail(DGS_ERR_INVALID_ARG, "alpha outside (0, 1]");
  if (!loss) return fail(DGS_ERR_INVALID_ARG, "loss is NULL");
  if (num_images > 0 && (!images || !targets || !target_of || num_targets < 1))
    return fail(DGS_ERR_INVALID_ARG, "images / targets / target_of missing");
  if ((num_expect > 0 && !expect) || (num_anchor > 0 && !anchor) || (num_mono > 0 && !mono) ||
      (num_temporal > 0 && !temporal))
    return fail(DGS_ERR_INVALID_ARG, "an index list is NULL");
  if (num_images == 0 && (num_expect > 0 || num_anchor > 0 || num_mono > 0 || num_temporal > 0))
    return fail(DGS_ERR_INVALID_ARG, "roles given for an empty batch");
  if (!scratch) return fail(DGS_ERR_INVALID_ARG, "scratch is NULL");
  if (((uintptr_t)scratch) & 255u) return fail(DGS_ERR_INVALID_ARG, "scratch not 256-byte aligned");
  const ObjLayout L = make_obj_layout(num_images, width, height, num_temporal);
  if (scratch_bytes < L.total) return fail(DGS_ERR_WORKSPACE, "scratch %zu bytes < %zu needed", scratch_bytes, L.total);
  ObjArgs a{};
  a.images = images;
  a.targets = targets;
  a.target_of = target_of;
  a.expect = expect;
  a.anchor = anchor;
  a.mono = mono;
  a.temporal = temporal;
  a.K = num_images;
  a.T = num_targets;
  a.width = width;
  a.height = height;
  a.n_expect = num_expect;
  a.n_anchor = num_anchor;
  a.n_mono = num_mono;
  a.n_temporal = num_temporal;
  a.bx = (int)ceil_div(width, 16);
  a.by = (int)ceil_div(height, 16);
  a.w = ObjWeights{w->lambda_ssim, w->lambda_c, w->alpha, w->lambda_t, w->lambda_m, w->lambda_a};
  a.loss = loss;
  a.distortion = distortion;
  a.grad = grad;
  a.hdr = at<ObjHeader>(scratch, L.header);
  a.dpart = at<double>(scratch, L.dpart);
  a.tpart = at<double>(scratch, L.tpart);
  a.tsum = at<double>(scratch, L.tsum);
  a.maps = at<float>(scratch, L.maps);
  a.coef = at<float>(scratch, L.coef);
  a.d = at<float>(scratch, L.d);
  a.cnt = at<int>(scratch, L.cnt);
  a.tcnt = at<int>(scratch, L.tcnt);
  a.tkey0 = at<uint32_t>(scratch, L.tkey0);
  a.tkey1 = at<uint32_t>(scratch, L.tkey1);
  a.tval0 = at<uint32_t>(scratch, L.tval0);
  a.tval1 = at<uint32_t>(scratch, L.tval1);
  a.thist = at<uint32_t>(scratch, L.thist);
  a.tparts = at<unsigned long long>(scratch, L.tparts);
  launch_objective(a, (hipStream_t)stream);
  return hip_check("objective launch");
}

size_t dgs_l1_scratch_bytes(int32_t num_images, int32_t width, int32_t height) {
  if (num_images < 0 || num_images > 65535 || width < 1 || height < 1 || width > 16384 || height > 16384) return 0;
  return l1_scratch_bytes(num_images, width, height);
}

static int check_l1(const float *images, int32_t num_images, int32_t width, int32_t height, const float *targets,
                    int32_t num_targets) {
  if (num_images < 0 || num_images > 65535) return fail(DGS_ERR_INVALID_ARG, "num_images %d outside 0..65535", num_images);
  if (width < 1 || height < 1 || width > 16384 || height > 16384)
    return fail(DGS_ERR_INVALID_ARG, "image size %dx%d outside 1..16384", width, height);
  if (num_images > 0 && (!images || !targets || num_targets < 1))
    return fail(DGS_ERR_INVALID_ARG, "images / targets missing");
  return DGS_OK;
}

int dgs_l1_loss(const float *images, int32_t num_images, int32_t width, int32_t height, const float *targets,
                int32_t num_targets, const int32_t *target_of, float *loss, void *scratch, size_t scratch_bytes,
                void *stream) {
  g_err.clear();
  int rc;
  if ((rc = check_l1(images, num_images, width, height, targets, num_targets))) return rc;
  if (!loss) return fail(DGS_ERR_INVALID_ARG, "loss is NULL");
  if (!scratch) return fail(DGS_ERR_INVALID_ARG, "scratch is NULL");
  if (((uintptr_t)scratch) & 255u) return fail(DGS_ERR_INVALID_ARG, "scratch not 256-byte aligned");
  const size_t need = l1_scratch_bytes(num_images, width, height);
  if (scratch_bytes < need) return fail(DGS_ERR_WORKSPACE, "scratch %zu bytes < %zu needed", scratch_bytes, need);
  launch_l1_loss(images, num_images, (int64_t)width * height * 3, targets, num_targets, target_of, loss, scratch,
                 (hipStream_t)stream);
  return hip_check("l1 loss launch");
}

int dgs_l1_loss_grad(const float *images, int32_t num_images, int32_t width, int32_t height, const float *targets,
                     int32_t num_targets, const int32_t *target_of, const float *dloss, float *grad, void *stream) {
  g_err.clear();
  int rc;
  if ((rc = check_l1(images, num_images, width, height, targets, num_targets))) return rc;
  if (num_images > 0 && !grad) return fail(DGS_ERR_INVALID_ARG, "grad is NULL");
  launch_l1_grad(images, num_images, (int64_t)width * height * 3, targets, num_targets, target_of, dloss, grad,
                 (hipStream_t)stream);
  return hip_check("l1 grad launch");
}

int dgs_objective_check(void *scratch, size_t scratch_bytes, void *stream) {
  g_err.clear();
  if (!scratch || scratch_bytes < sizeof(ObjHeader)) return fail(DGS_ERR_INVALID_ARG, "objective scratch missing");
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = refuse_capture(st, "dgs_objective_check"))) return rc;
  ObjHeader h;
  if (hipMemcpyAsync(&h, scratch, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return hip_check("objective check copy");
  if (h.bad) return fail(DGS_ERR_INVALID_ARG, "an index in the objective's lists or target_of is out of range");
  return hip_check("objective check");
}

}  // extern "C"
