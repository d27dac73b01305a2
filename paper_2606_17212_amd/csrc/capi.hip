// C ABI of the renderer: argument validation, workspace layout and the launch
// sequence of each entry point.  Declarations and contracts: include/dgs.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "../../include/dgs.h"
#include "common.h"
#include "kernels.h"

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
  call->L = make_layout(scene->n, P, call->tiling.tiles_x, call->tiling.tiles_y, states->num_states, cap);
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

// Projection, depth sort, instance count and offsets.  `list_mode`: only the
// Gaussians listed in ws.list (count in header.n_active) take part.
void project_and_count(const Call &cl, void *ws, bool list_mode, hipStream_t st) {
  const Layout &L = cl.L;
  Header *h = at<Header>(ws, L.header);
  const int n = cl.s.n;
  const uint32_t *list = list_mode ? at<uint32_t>(ws, L.present) : nullptr;
  const unsigned *nact = list_mode ? &h->n_active : nullptr;
  launch_geometry(cl.s, cl.c, cl.t, list, nact, n, at<float4>(ws, L.rec0), at<float4>(ws, L.rec1),
                  at<float4>(ws, L.rec2), at<uint2>(ws, L.rect), at<uint2>(ws, L.pbox),
                  at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), st);
  // depth keys: 32 bits, 4 passes -> result back in dkey0/dval0
  launch_radix_sort(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), at<uint32_t>(ws, L.dkey1),
                    at<uint32_t>(ws, L.dval1), nact, 0, n, 0, 32, at<uint32_t>(ws, L.hist),
                    at<unsigned long long>(ws, L.part), st);
  launch_count(at<uint32_t>(ws, L.dkey0), at<uint32_t>(ws, L.dval0), at<uint2>(ws, L.rect), nact, n,
               at<uint32_t>(ws, L.cnt), st);
  // offsets go to dkey1 (free after the depth sort)
  launch_scan_u32(at<uint32_t>(ws, L.cnt), at<uint32_t>(ws, L.dkey1), n, at<unsigned long long>(ws, L.part),
                  &h->instances, st);
}

// Emission, tile sort and ranges; returns the sorted Gaussian ids.
const uint32_t *emit_and_sort(const Call &cl, void *ws, bool list_mode, int64_t cap, hipStream_t st) {
  const Layout &L = cl.L;
  Header *h = at<Header>(ws, L.header);
  const int n = cl.s.n;
  const unsigned *nact = list_mode ? &h->n_active : nullptr;
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

const uint32_t *sorted_vals(const Call &cl, void *ws) {
  const int passes = (cl.tiling.tile_bits + 7) / 8;
  return (passes & 1) ? at<uint32_t>(ws, cl.L.tval1) : at<uint32_t>(ws, cl.L.tval0);
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
  dgs_states st0 = *states;
  st0.num_states = 0;  // no per-state buffers needed
  Call cl;
  int rc = prepare(scene, cam, &st0, tun, ws, ws_bytes, 0, 0, &cl);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  Header *h = at<Header>(ws, cl.L.header);
  launch_clear_header(h, 0ull, st);
  project_and_count(cl, ws, false, st);
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
  Header *h = at<Header>(ws, cl.L.header);
  launch_clear_header(h, (unsigned long long)cap, st);
  project_and_count(cl, ws, false, st);
  emit_and_sort(cl, ws, false, cap, st);
  launch_plhist(scene->packet_layer, cl.s.n, cl.P, at<uint32_t>(ws, cl.L.plhist), st);
  launch_tile_order(at<uint2>(ws, cl.L.ranges), cl.tiling.tiles, at<uint32_t>(ws, cl.L.tile_order), st);
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
  launch_visbits(states->codes, order, W, cl.P, S, visbits, st);
  CompositeArgs a = composite_args(cl, ws, sorted_vals(cl, ws), states, visbits, groups);
  a.state_order = order;
  a.launch_states = W;
  a.image = image;
  a.tfinal = tfinal;
  a.reference = reference;
  a.psnr_part = at<float>(ws, cl.L.psnr_part);
  a.counters = counters;
  a.queues = at<unsigned int>(ws, cl.L.queues);
  const int launch = !tun ? 0 : (tun->flags & DGS_TUNE_PERSISTENT) ? 1 : (tun->flags & DGS_TUNE_GRID) ? 2 : 0;
  if (launch_composite(a, S, cl.tiling.tw, cl.tiling.th, mode, launch, st))
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
    launch_clear_header(h, (unsigned long long)cap, st);
    // compaction of the delivered Gaussians (flags -> scan -> scatter)
    launch_present_flags(states->codes + (int64_t)w * cl.P, scene->packet_layer, n, cl.P,
                         at<uint32_t>(ws, cl.L.cnt), st);
    launch_scan_u32(at<uint32_t>(ws, cl.L.cnt), at<uint32_t>(ws, cl.L.dkey1), n,
                    at<unsigned long long>(ws, cl.L.part), &h->instances, st);
    launch_present_scatter(at<uint32_t>(ws, cl.L.cnt), at<uint32_t>(ws, cl.L.dkey1), n,
                           at<uint32_t>(ws, cl.L.present), &h->instances, h, st);
    project_and_count(cl, ws, true, st);
    const uint32_t *vals = emit_and_sort(cl, ws, true, cap, st);
    launch_tile_order(at<uint2>(ws, cl.L.ranges), cl.tiling.tiles, at<uint32_t>(ws, cl.L.tile_order), st);
    CompositeArgs a = composite_args(cl, ws, vals, states, nullptr, 1);
    a.image = image;
    a.tfinal = tfinal;
    a.state_offset = w;
    a.launch_states = 1;
    if (launch_composite(a, 1, cl.tiling.tw, cl.tiling.th, 0, 2, st))
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
                                 !grad->color || (scene->rank > 0 && !grad->temporal))))
    return fail(DGS_ERR_INVALID_ARG, "gradient pointer is NULL");
  const int W = states->num_states;
  if (W > 0 && (!image || !grad_image)) return fail(DGS_ERR_INVALID_ARG, "image / grad_image is NULL");
  hipStream_t st = (hipStream_t)stream;
  const int n = cl.s.n;
  float *g2d = at<float>(ws, cl.L.grad2d);
  launch_fill_f32(g2d, (int64_t)9 * n, 0.0f, st);
  if (W > 0) {
    const int S = group_size(tun, W, 8);
    const int groups = (W + S - 1) / S;
    uint32_t *visbits = at<uint32_t>(ws, cl.L.visbits);
    uint32_t *order = at<uint32_t>(ws, cl.L.state_order);
    launch_state_order(states->codes, at<uint32_t>(ws, cl.L.plhist), W, cl.P, at<uint32_t>(ws, cl.L.state_cnt),
                       order, st);
    launch_visbits(states->codes, order, W, cl.P, S, visbits, st);
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
                      grad->color, grad->temporal, st);
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

int dgs_check(void *ws, size_t ws_bytes, int64_t *instances, void *stream) {
  g_err.clear();
  if (!ws || ws_bytes < sizeof(Header)) return fail(DGS_ERR_INVALID_ARG, "workspace missing");
  hipStream_t st = (hipStream_t)stream;
  Header hh;
  if (hipMemcpyAsync(&hh, ws, sizeof(Header), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return hip_check("check copy");
  if (instances) *instances = (int64_t)hh.instances;
  if (hh.overflow)
    return fail(DGS_ERR_OVERFLOW, "%llu instances exceed capacity %llu", hh.instances, hh.capacity);
  return hip_check("check");
}

}  // extern "C"
