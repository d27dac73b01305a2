/*
 * Reference renderer for a dynamic Gaussian scene under incomplete delivery
 * states.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU
 * baseline leg of the bench call it; the renderer library never links, loads
 * or calls anything here, and nothing here is shared with it.
 *
 * What is computed (plain definitions, FP64 unless stated):
 *
 *  - Delivery decode: Gaussian i (packet p_i, layer l_i) is present in state w
 *    iff l_i < codes[w][p_i]; codes are post-closure cluster/context masks with
 *    a delivered prefix depth (Sec. 4, Sec. 3 "one base + three refinements").
 *  - Deformation, Eq. (1) of Sec. 3:
 *        mu_i = A_c [mubar_i; 1] + sum_r b_r q_{i,r} + o_i,
 *    o_i = the delivered residual levels (delta terms) at the render time, or
 *    0 when the scene carries none.
 *  - Projection: camera-frame mean, covariance R diag(e^{2s}) R^T seen through
 *    the world->camera rotation, local affine (EWA) Jacobian with its x/z and
 *    y/z arguments clamped to 1.3x the half field of view, +0.3 px^2 on the
 *    2D covariance diagonal, conic = inverse 2D covariance.
 *  - Opacity sigmoid(logit); colour RGB, or degree-1 real SH with
 *    Condon-Shortley phase + 0.5, clamped at 0, evaluated along the direction
 *    from the camera centre to the deformed mean.
 *  - Per pixel (centre at +0.5) and state: the present, un-culled Gaussians
 *    with alpha = min(0.99, o exp(-q/2)) >= 1/255, ordered by (FP32 camera
 *    depth bits, index), composited front to back, C += T alpha c,
 *    T *= (1 - alpha); compositing stops right after the first Gaussian that
 *    leaves T < 1e-4; finally C += T * background.
 *
 * The sort order and the culling (depth <= near plane) are integer decisions
 * taken in FP32 by a mirror whose arithmetic order is fixed below
 * (or_mirror_f32); the tile rectangles used by a tiled renderer are also
 * decided there.  Both sides of a parity check take these decisions in FP32.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared
 * (no FMA contraction and no excess precision: x86-64 SSE float arithmetic).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n;
  int32_t rank;
  int32_t sh_degree;
  int32_t num_packets;
  int32_t num_contexts;
  const float *mean;          /* [3][n] */
  const float *log_scale;     /* [3][n] */
  const float *quat;          /* [4][n] (w,x,y,z) */
  const float *opacity_logit; /* [n] */
  const float *color;         /* [3][n] rgb or [12][n] SH-1, row = coef*3 + channel */
  const float *temporal;      /* [3*rank][n], row = r*3 + axis */
  const uint16_t *packet_layer; /* [n] (packet << 2) | layer */
  const float *cluster_affine;  /* [C][12] row-major 3x4, or NULL (identity) */
  const float *offset;          /* [3][n] position residual added after the deformation, or NULL */
} or_scene;

typedef struct {
  float R[9];  /* world -> camera rotation, row-major */
  float t[3];
  float fx, fy, cx, cy, near_z;
  int32_t width, height;
} or_camera;

/* ------------------------------------------------------------------------ */
/* FP32 mirror                                                              */
/* ------------------------------------------------------------------------ */

/* e^x in FP32 by Cody & Waite (1980) argument reduction, e^x = 2^n e^r with
 * n = rint(x log2 e), r = (x - n ln2_hi) - n ln2_lo, and e^r from the
 * degree-7 Taylor polynomial in Horner form.  Every operation is a single
 * correctly rounded IEEE operation, so the value is reproducible bit for bit
 * by any implementation that follows the same steps. */
float or_exp_f32(float x) {
  const float log2e = 0x1.715476p+0f;
  const float ln2_hi = 0x1.62e4p-1f;
  const float ln2_lo = 0x1.7f7d1cp-20f;
  float n = rintf(x * log2e);
  float r = (x - n * ln2_hi) - n * ln2_lo;
  float p = 0x1.a01a02p-13f;          /* 1/7! */
  p = p * r + 0x1.6c16c2p-10f;        /* 1/6! */
  p = p * r + 0x1.111112p-7f;         /* 1/5! */
  p = p * r + 0x1.555556p-5f;         /* 1/4! */
  p = p * r + 0x1.555556p-3f;         /* 1/3! */
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  return ldexpf(p, (int)n);
}

static inline float clampf(float x, float lo, float hi) {
  return fminf(fmaxf(x, lo), hi);
}

/* Per Gaussian FP32 quantities that decide integers:
 *   out_f [6][n]: z32, u, v, a, b, c   (2D covariance [[a,b],[b,c]] incl. +0.3)
 *   rect  [4][n]: tile x0, y0, x1, y1 (half-open) -- empty when culled
 *   valid [n]   : 1 unless culled (z32 <= near, or det <= 0)
 * Arithmetic order (each product, quotient, sum rounded separately):
 *   mu_k  = ((A_k0 m0 + A_k1 m1) + A_k2 m2) + A_k3   (or m_k with no affine),
 *           then mu_k += b_r q_{r,k} for r = 0..R-1, then mu_k += o_k (offset)
 *   P_k   = ((R_k0 mu0 + R_k1 mu1) + R_k2 mu2) + t_k;  (X,Y,Z) = P
 *   xz = X/Z, yz = Y/Z, u = fx xz + cx, v = fy yz + cy
 *   limx = (0.65 W)/fx, limy = (0.65 H)/fy, txz = clamp(xz), tyz = clamp(yz)
 *   j00 = fx/Z, j02 = -(fx txz)/Z, j11 = fy/Z, j12 = -(fy tyz)/Z
 *   quaternion: n2 = ((w w + x x) + y y) + z z, r = sqrt(n2), each / r;
 *     Rq00 = 1 - 2(yy + zz), Rq01 = 2(xy - wz), Rq02 = 2(xz + wy),
 *     Rq10 = 2(xy + wz), Rq11 = 1 - 2(xx + zz), Rq12 = 2(yz - wx),
 *     Rq20 = 2(xz - wy), Rq21 = 2(yz + wx), Rq22 = 1 - 2(xx + yy)
 *   vk = exp_f32(2 s_k)
 *   M0j = j00 Rcw0j + j02 Rcw2j, M1j = j11 Rcw1j + j12 Rcw2j
 *   Vij = (Mi0 Rq0j + Mi1 Rq1j) + Mi2 Rq2j
 *   a = (((V00 V00) v0 + (V01 V01) v1) + (V02 V02) v2) + 0.3
 *   b = ((V00 V10) v0 + (V01 V11) v1) + (V02 V12) v2
 *   c = (((V10 V10) v0 + (V11 V11) v1) + (V12 V12) v2) + 0.3
 *   det = a c - b b
 *   A = c / det, B = -b / det, C = a / det;
 *   A' = kA A, B' = kB B, C' = kA C with kA = fl32(-log2(e)/2), kB = fl32(-log2(e))
 *   ex = sqrt(11.1 a), ey = sqrt(11.1 c)
 *   x0 = clamp(floor((u - ex)/TW), 0, tiles_x), x1 = clamp(floor((u + ex)/TW) + 1, 0, tiles_x)
 *   (y likewise with TH, tiles_y); TW, TH powers of two.
 */
static void mirror_one(const or_scene *s, const or_camera *cam, const float *basis,
                       int tile_w, int tile_h, int64_t i, float *f9, int32_t *r4,
                       int32_t *valid) {
  const int64_t n = s->n;
  float m0 = s->mean[i], m1 = s->mean[n + i], m2 = s->mean[2 * n + i];
  float mu[3];
  int cl = (int)(s->packet_layer[i] >> 2) / s->num_contexts;
  for (int k = 0; k < 3; ++k) {
    if (s->cluster_affine) {
      const float *A = s->cluster_affine + 12 * cl + 4 * k;
      mu[k] = ((A[0] * m0 + A[1] * m1) + A[2] * m2) + A[3];
    } else {
      mu[k] = (k == 0) ? m0 : (k == 1) ? m1 : m2;
    }
    for (int r = 0; r < s->rank; ++r) mu[k] = mu[k] + basis[r] * s->temporal[(3 * r + k) * n + i];
    if (s->offset) mu[k] = mu[k] + s->offset[k * n + i];
  }
  float P[3];
  for (int k = 0; k < 3; ++k)
    P[k] = ((cam->R[3 * k] * mu[0] + cam->R[3 * k + 1] * mu[1]) + cam->R[3 * k + 2] * mu[2]) + cam->t[k];
  float X = P[0], Y = P[1], Z = P[2];
  float xz = X / Z, yz = Y / Z;
  float u = cam->fx * xz + cam->cx, v = cam->fy * yz + cam->cy;
  float limx = (0.65f * (float)cam->width) / cam->fx;
  float limy = (0.65f * (float)cam->height) / cam->fy;
  float txz = clampf(xz, -limx, limx), tyz = clampf(yz, -limy, limy);
  float j00 = cam->fx / Z, j02 = -(cam->fx * txz) / Z;
  float j11 = cam->fy / Z, j12 = -(cam->fy * tyz) / Z;

  float qw = s->quat[i], qx = s->quat[n + i], qy = s->quat[2 * n + i], qz = s->quat[3 * n + i];
  float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  float nr = sqrtf(n2);
  float w = qw / nr, x = qx / nr, y = qy / nr, z = qz / nr;
  float Rq[9];
  Rq[0] = 1.0f - 2.0f * (y * y + z * z);
  Rq[1] = 2.0f * (x * y - w * z);
  Rq[2] = 2.0f * (x * z + w * y);
  Rq[3] = 2.0f * (x * y + w * z);
  Rq[4] = 1.0f - 2.0f * (x * x + z * z);
  Rq[5] = 2.0f * (y * z - w * x);
  Rq[6] = 2.0f * (x * z - w * y);
  Rq[7] = 2.0f * (y * z + w * x);
  Rq[8] = 1.0f - 2.0f * (x * x + y * y);

  float vs[3];
  for (int k = 0; k < 3; ++k) vs[k] = or_exp_f32(2.0f * s->log_scale[k * n + i]);

  float M[6];
  for (int j = 0; j < 3; ++j) {
    M[j] = j00 * cam->R[j] + j02 * cam->R[6 + j];
    M[3 + j] = j11 * cam->R[3 + j] + j12 * cam->R[6 + j];
  }
  float V[6];
  for (int r = 0; r < 2; ++r)
    for (int j = 0; j < 3; ++j)
      V[3 * r + j] = (M[3 * r] * Rq[j] + M[3 * r + 1] * Rq[3 + j]) + M[3 * r + 2] * Rq[6 + j];
  float a = (((V[0] * V[0]) * vs[0] + (V[1] * V[1]) * vs[1]) + (V[2] * V[2]) * vs[2]) + 0.3f;
  float b = ((V[0] * V[3]) * vs[0] + (V[1] * V[4]) * vs[1]) + (V[2] * V[5]) * vs[2];
  float c = (((V[3] * V[3]) * vs[0] + (V[4] * V[4]) * vs[1]) + (V[5] * V[5]) * vs[2]) + 0.3f;
  float det = a * c - b * b;
  const float kA = -0x1.715476p-1f, kB = -0x1.715476p+0f; /* -log2(e)/2, -log2(e) in FP32 */
  float cA = c / det, cB = -b / det, cC = a / det;

  int ok = (Z > cam->near_z) && (det > 0.0f);
  f9[0] = Z; f9[1] = u; f9[2] = v; f9[3] = a; f9[4] = b; f9[5] = c;
  f9[6] = kA * cA; f9[7] = kB * cB; f9[8] = kA * cC;
  *valid = ok;
  r4[0] = r4[1] = r4[2] = r4[3] = 0;
  if (!ok) return;
  int tiles_x = (cam->width + tile_w - 1) / tile_w;
  int tiles_y = (cam->height + tile_h - 1) / tile_h;
  float itw = 1.0f / (float)tile_w, ith = 1.0f / (float)tile_h; /* exact: powers of two */
  float ex = sqrtf(11.1f * a), ey = sqrtf(11.1f * c);
  float x0 = clampf(floorf((u - ex) * itw), 0.0f, (float)tiles_x);
  float x1 = clampf(floorf((u + ex) * itw) + 1.0f, 0.0f, (float)tiles_x);
  float y0 = clampf(floorf((v - ey) * ith), 0.0f, (float)tiles_y);
  float y1 = clampf(floorf((v + ey) * ith) + 1.0f, 0.0f, (float)tiles_y);
  r4[0] = (int32_t)x0; r4[1] = (int32_t)y0; r4[2] = (int32_t)x1; r4[3] = (int32_t)y1;
}

int or_mirror_f32(const or_scene *s, const or_camera *cam, const float *basis,
                  int tile_w, int tile_h, float *out_f /*[9][n]*/, int32_t *rect /*[4][n]*/,
                  int32_t *valid /*[n]*/) {
  const int64_t n = s->n;
  if (tile_w <= 0 || tile_h <= 0 || (tile_w & (tile_w - 1)) || (tile_h & (tile_h - 1))) return 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    float f9[9];
    int32_t r4[4], ok;
    mirror_one(s, cam, basis, tile_w, tile_h, i, f9, r4, &ok);
    for (int k = 0; k < 9; ++k) out_f[k * n + i] = f9[k];
    for (int k = 0; k < 4; ++k) rect[k * n + i] = r4[k];
    valid[i] = ok;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* FP64 geometry (the definition)                                            */
/* ------------------------------------------------------------------------ */

enum { G_U, G_V, G_A2, G_B2, G_C2, G_CA, G_CB, G_CC, G_O, G_R, G_G, G_B, G_X, G_Y, G_Z, G_NF };

static const double SH_C0 = 0.28209479177387814;  /* 1 / (2 sqrt(pi)) */
static const double SH_C1 = 0.4886025119029199;   /* sqrt(3) / (2 sqrt(pi)) */

static void mat3_mul(const double *A, const double *B, double *C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = acc;
    }
}

static void geometry_one(const or_scene *s, const or_camera *cam, const float *basis,
                         int64_t i, double *g) {
  const int64_t n = s->n;
  double m[3] = {s->mean[i], s->mean[n + i], s->mean[2 * n + i]};
  double mu[3];
  int cl = (int)(s->packet_layer[i] >> 2) / s->num_contexts;
  for (int k = 0; k < 3; ++k) {
    if (s->cluster_affine) {
      const float *A = s->cluster_affine + 12 * cl + 4 * k;
      mu[k] = (double)A[0] * m[0] + (double)A[1] * m[1] + (double)A[2] * m[2] + (double)A[3];
    } else {
      mu[k] = m[k];
    }
    for (int r = 0; r < s->rank; ++r) mu[k] += (double)basis[r] * (double)s->temporal[(3 * r + k) * n + i];
    if (s->offset) mu[k] += (double)s->offset[k * n + i];
  }
  double Rc[9];
  for (int k = 0; k < 9; ++k) Rc[k] = cam->R[k];
  double P[3];
  for (int k = 0; k < 3; ++k)
    P[k] = Rc[3 * k] * mu[0] + Rc[3 * k + 1] * mu[1] + Rc[3 * k + 2] * mu[2] + (double)cam->t[k];
  double X = P[0], Y = P[1], Z = P[2];
  double fx = cam->fx, fy = cam->fy;

  /* rotation of the normalised quaternion (w, x, y, z) */
  double q[4] = {s->quat[i], s->quat[n + i], s->quat[2 * n + i], s->quat[3 * n + i]};
  double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  /* Sigma = Rq diag(e^{2s}) Rq^T */
  double RS[9], RqT[9], Sig[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      RS[3 * r + c] = Rq[3 * r + c] * exp(2.0 * (double)s->log_scale[c * n + i]);
      RqT[3 * r + c] = Rq[3 * c + r];
    }
  mat3_mul(RS, RqT, Sig);
  /* camera-frame covariance Rc Sigma Rc^T */
  double RcT[9], T1[9], Sc[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) RcT[3 * r + c] = Rc[3 * c + r];
  mat3_mul(Rc, Sig, T1);
  mat3_mul(T1, RcT, Sc);
  /* local affine Jacobian with clamped x/z, y/z */
  double limx = 1.3 * (double)cam->width / (2.0 * fx);
  double limy = 1.3 * (double)cam->height / (2.0 * fy);
  double tx = X / Z, ty = Y / Z;
  if (tx < -limx) tx = -limx;
  if (tx > limx) tx = limx;
  if (ty < -limy) ty = -limy;
  if (ty > limy) ty = limy;
  double J[6] = {fx / Z, 0.0, -fx * tx / Z, 0.0, fy / Z, -fy * ty / Z};
  double S2[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += J[3 * r + k] * Sc[3 * k + l] * J[3 * c + l];
      S2[2 * r + c] = acc;
    }
  double a = S2[0] + 0.3, b = S2[1], c = S2[3] + 0.3;
  double det = a * c - b * b;
  g[G_A2] = a; g[G_B2] = b; g[G_C2] = c;
  g[G_CA] = c / det; g[G_CB] = -b / det; g[G_CC] = a / det;
  g[G_U] = fx * X / Z + (double)cam->cx;
  g[G_V] = fy * Y / Z + (double)cam->cy;
  g[G_O] = 1.0 / (1.0 + exp(-(double)s->opacity_logit[i]));
  if (s->sh_degree == 0) {
    for (int ch = 0; ch < 3; ++ch) g[G_R + ch] = s->color[ch * n + i];
  } else {
    /* camera centre C = -Rc^T t; direction from C to the deformed mean */
    double C[3];
    for (int k = 0; k < 3; ++k)
      C[k] = -(Rc[k] * cam->t[0] + Rc[3 + k] * cam->t[1] + Rc[6 + k] * cam->t[2]);
    double d[3] = {mu[0] - C[0], mu[1] - C[1], mu[2] - C[2]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int k = 0; k < 3; ++k) d[k] /= dn;
    for (int ch = 0; ch < 3; ++ch) {
      double k0 = s->color[(0 * 3 + ch) * n + i], k1 = s->color[(1 * 3 + ch) * n + i];
      double k2 = s->color[(2 * 3 + ch) * n + i], k3 = s->color[(3 * 3 + ch) * n + i];
      double val = 0.5 + SH_C0 * k0 + SH_C1 * (-d[1] * k1 + d[2] * k2 - d[0] * k3);
      g[G_R + ch] = val > 0.0 ? val : 0.0;
    }
  }
  g[G_X] = X; g[G_Y] = Y; g[G_Z] = Z;
}

int or_geometry_f64(const or_scene *s, const or_camera *cam, const float *basis,
                    double *out /*[G_NF][n]*/) {
  const int64_t n = s->n;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double g[G_NF];
    geometry_one(s, cam, basis, i, g);
    for (int k = 0; k < G_NF; ++k) out[k * n + i] = g[k];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint32_t zbits;
  int32_t id;
  double alpha; /* FP64 alpha (the definition) */
  double rho;   /* bound on |alpha_32 / alpha - 1| of an FP32 renderer */
  int amb;      /* an FP32 renderer may take the other side of the 1/255 skip */
} cand_t;

static int cand_cmp(const void *pa, const void *pb) {
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  if (a->zbits != b->zbits) return a->zbits < b->zbits ? -1 : 1;
  return (a->id > b->id) - (a->id < b->id);
}

#define ALPHA_MIN (1.0 / 255.0)
#define T_STOP 1e-4

/*
 * Ambiguity budget: where an FP32 renderer may legitimately take the other
 * branch of a discrete decision, and by how much its image may then differ.
 *
 * The FP32 renderer evaluates, per (Gaussian, pixel), the base-2 exponent
 *     q' = A' dx^2 + B' dx dy + C' dy^2 + l,   dx = u - (px + 0.5), dy likewise,
 * from its FP32 record (u, v, A', B', C') -- the values or_mirror_f32 computes,
 * in the same operation order -- and its FP32 log2-opacity l; it skips the
 * pair when q' < fl32(log2(1/255)), uses alpha = min(fl32(0.99), 2^q') (the
 * hardware base-2 exponential), then T alpha and T - T alpha, each rounded
 * once, and stops when T - T alpha < fl32(1e-4).
 *
 * Bounds (EPS = 2^-24, the FP32 unit roundoff):
 *  - qg = the exponent from the mirror's FP32 record and the FP64 log2(o),
 *    evaluated in FP64 (exact to ~1e-16).  The renderer's q' differs from qg
 *    by at most E = EVAL_ROUNDINGS EPS S + DLO: the rounding of dx and of the
 *    five products / fused adds of the quadratic form, each at most EPS of a
 *    partial sum bounded by S = |A'| dx^2 + |B' dx dy| + |C'| dy^2 + |l|,
 *    plus DLO, the error of the record's log2-opacity (hardware exp and log;
 *    the GPU tests check every record against DLO).
 *  - skip: the definition skips iff alpha < 1/255; the renderer's decision
 *    can differ only if qg - E < fl32(log2(1/255)) <= qg + E disagrees with
 *    it.  A skip that may flip adds 2 T alpha M (with or without the
 *    Gaussian the colour differs by T alpha (c - colour behind it)) and lets
 *    T differ by the factor 1 - alpha (relative alpha / (1 - alpha)).
 *  - alpha: |alpha_32 / alpha - 1| <= rho = (2^(|qg - q64| + E) - 1)(1 + XR) + XR,
 *    with q64 = log2 of the FP64 alpha and XR = 2^-22 for the hardware 2^x
 *    (1 ulp, doubled); rho = XR where both sides surely take the 0.99 cap
 *    (|fl32(0.99) - 0.99| < XR).
 *  - transmittance: after a composited alpha the relative error of T grows
 *    multiplicatively by (1 + EPS)(1 + (alpha / (1 - alpha)) ((1 + rho)(1 + EPS) - 1))
 *    (rounding of T alpha and of T - T alpha, and the alpha error).
 *  - stop: the definition stops iff T_after < 1e-4; the renderer's T lies in
 *    T_after (1 +- relT); a stop that may flip adds 2 T_after (1 + relT) M
 *    (what the rest of the list and the background can contribute).
 *  M = max |colour| over the pixel's candidates and |background|, + 2^-16 for
 *  the FP32 colour.
 */
#define EPS32 (1.0 / 16777216.0)
#define EVAL_ROUNDINGS 8.0
#define DLO (1.0 / 65536.0)
#define EXP_REL (1.0 / 4194304.0)

/*
 * Render npix pixels (pix_xy = x,y pairs; NULL = every pixel, row-major) for
 * num_states states.  Outputs, indexed [w][k]:
 *   image  [W][npix][3]  composited colour incl. background
 *   tfinal [W][npix]     transmittance after the last composited Gaussian
 *   budget [W][npix]     ambiguity budget (above): the largest change an FP32
 *                        renderer may legitimately show at the pixel
 *   ncomp  [W][npix]     number of composited Gaussians (present pairs)
 */
int or_render(const or_scene *s, const or_camera *cam, const float *basis, int num_states,
              const uint8_t *codes /*[W][P]*/, const float *bg, int64_t npix,
              const int32_t *pix_xy, double *image, double *tfinal, double *budget,
              int32_t *ncomp) {
  const int64_t n = s->n;
  const int P = s->num_packets;
  double *geo = (double *)malloc(sizeof(double) * G_NF * (size_t)(n > 0 ? n : 1));
  float *mf = (float *)malloc(sizeof(float) * 9 * (size_t)(n > 0 ? n : 1));
  int32_t *rect = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(n > 0 ? n : 1));
  int32_t *valid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!geo || !mf || !rect || !valid) {
    free(geo); free(mf); free(rect); free(valid);
    return 2;
  }
  or_geometry_f64(s, cam, basis, geo);
  or_mirror_f32(s, cam, basis, 16, 16, mf, rect, valid);
  const int Wd = cam->width;
  double bgd[3] = {bg[0], bg[1], bg[2]};
  double bgmax = fmax(fabs(bgd[0]), fmax(fabs(bgd[1]), fabs(bgd[2])));
  const double log2e = 1.0 / log(2.0);
  const double qskip32 = (double)(float)(-log2(255.0)); /* the FP32 renderer's skip threshold */
  const double tstop32 = (double)1e-4f;                 /* and its stop threshold */
  const double log2cap32 = log2((double)0.99f);         /* 2^q' above this: alpha_32 = fl32(0.99) */
  int err = 0;

#pragma omp parallel
  {
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
    if (!cand) {
#pragma omp atomic write
      err = 2;
    }
#pragma omp for schedule(dynamic, 8)
    for (int64_t k = 0; k < npix; ++k) {
      if (!cand) continue;
      int px = pix_xy ? pix_xy[2 * k] : (int)(k % Wd);
      int py = pix_xy ? pix_xy[2 * k + 1] : (int)(k / Wd);
      double cxp = px + 0.5, cyp = py + 0.5;
      int64_t nc = 0;
      double colmax = bgmax;
      for (int64_t i = 0; i < n; ++i) {
        if (!valid[i]) continue;
        double dx = geo[G_U * n + i] - cxp, dy = geo[G_V * n + i] - cyp;
        double q = geo[G_CA * n + i] * dx * dx + 2.0 * geo[G_CB * n + i] * dx * dy +
                   geo[G_CC * n + i] * dy * dy;
        double o = geo[G_O * n + i];
        double al = o * exp(-0.5 * q);
        if (al > 0.99) al = 0.99;
        /* the FP32 renderer's exponent, from the mirror's record */
        double lo = log2(o);
        double fx = (double)mf[1 * n + i] - cxp, fy = (double)mf[2 * n + i] - cyp;
        double tA = (double)mf[6 * n + i] * fx * fx, tB = (double)mf[7 * n + i] * fx * fy;
        double tC = (double)mf[8 * n + i] * fy * fy;
        double qg = tA + tB + tC + lo;
        double E = EVAL_ROUNDINGS * EPS32 * (fabs(tA) + fabs(tB) + fabs(tC) + fabs(lo)) + DLO;
        int skip = al < ALPHA_MIN;
        int amb = skip ? (qg + E >= qskip32) : (qg - E < qskip32);
        if (skip && !amb) continue;
        double q64 = lo - 0.5 * log2e * q; /* log2 of the uncapped FP64 alpha */
        uint32_t zb;
        memcpy(&zb, &mf[i], 4);
        cand[nc].zbits = zb;
        cand[nc].id = (int32_t)i;
        cand[nc].alpha = al;
        /* both sides surely capped: alpha_32 = fl32(0.99) against 0.99 */
        int capped = (q64 >= log2(0.99)) && (qg - E - EXP_REL > log2cap32);
        cand[nc].rho = capped ? EXP_REL : (exp2(fabs(qg - q64) + E) - 1.0) * (1.0 + EXP_REL) + EXP_REL;
        cand[nc].amb = amb;
        ++nc;
        for (int ch = 0; ch < 3; ++ch) colmax = fmax(colmax, fabs(geo[(G_R + ch) * n + i]));
      }
      qsort(cand, (size_t)nc, sizeof(cand_t), cand_cmp);
      const double M = colmax + DLO;
      for (int w = 0; w < num_states; ++w) {
        const uint8_t *cw = codes + (int64_t)w * P;
        double T = 1.0, C[3] = {0.0, 0.0, 0.0}, B = 0.0, relT = 0.0;
        int32_t cnt = 0;
        for (int64_t j = 0; j < nc; ++j) {
          int32_t i = cand[j].id;
          uint16_t pl = s->packet_layer[i];
          if ((int)(pl & 3u) >= (int)cw[pl >> 2]) continue; /* not delivered */
          double al = cand[j].alpha;
          double odds = al / (1.0 - al);
          if (cand[j].amb) {
            B += 2.0 * T * al * M;
            relT = (1.0 + relT) * (1.0 + odds) - 1.0;
          }
          if (al < ALPHA_MIN) continue;
          for (int ch = 0; ch < 3; ++ch) C[ch] += T * al * geo[(G_R + ch) * n + i];
          double Ta = T * (1.0 - al);
          ++cnt;
          relT = (1.0 + relT) * (1.0 + EPS32) *
                     (1.0 + odds * ((1.0 + cand[j].rho) * (1.0 + EPS32) - 1.0)) - 1.0;
          int stop = Ta < T_STOP;
          int amb_stop = stop ? (Ta * (1.0 + relT) >= tstop32) : (Ta * (1.0 - relT) < tstop32);
          if (amb_stop) B += 2.0 * Ta * (1.0 + relT) * M;
          T = Ta;
          if (stop) break;
        }
        for (int ch = 0; ch < 3; ++ch) C[ch] += T * bgd[ch];
        int64_t o = (int64_t)w * npix + k;
        for (int ch = 0; ch < 3; ++ch) image[3 * o + ch] = C[ch];
        if (tfinal) tfinal[o] = T;
        if (budget) budget[o] = B;
        if (ncomp) ncomp[o] = cnt;
      }
    }
    free(cand);
  }
  free(geo); free(mf); free(rect); free(valid);
  return err;
}

/* ------------------------------------------------------------------------
 * Delivery-state sampler (Sec. 4: a training world samples erasures from an
 * IID process and a Gilbert-Elliott burst process; dependencies are enforced
 * after delivery and turned into cluster-layer masks).
 *
 * Every (packet p, layer l) is one datagram, sent layer-major (all base
 * layers, then every first refinement, ...): slot s = l P + p.  The channel
 * of world w is a two-state Markov chain (good / bad) over the slots: the
 * datagram of slot s is erased with the loss probability of the current
 * state, then the chain moves (good -> bad with p_gb, bad -> good with p_bg);
 * the first state is bad with probability p_start_bad.  Datagrams of slots
 * >= deadline arrive too late (deadline < 0: none).  Layer l of packet p is
 * usable when layers 0..l all arrived, so the state's code for p is the
 * number of leading arrived layers.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
 * the 64-bit seed, counter (s / 2, w, 0x44475331, 0) for slot s: outputs
 * (x0, x1) serve even slots and (x2, x3) odd ones as (erasure, transition)
 * draws; counter (0xffffffff, w, 0x44475331, 0) output x0 draws the first
 * state.  An event of probability p happens when the draw is below
 * floor(p 2^32) (p <= 0: never; p >= 1: always).
 * ---------------------------------------------------------------------- */
typedef struct {
  float p_gb, p_bg, loss_good, loss_bad, p_start_bad;
  int32_t deadline;
} or_channel;

static const uint32_t OR_SAMPLER_TAG = 0x44475331u;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static uint64_t or_threshold(float p) {
  if (!(p > 0.0f)) return 0;
  if (p >= 1.0f) return (uint64_t)1 << 32;
  return (uint64_t)floor((double)p * 4294967296.0);
}

int or_sample_states(const or_channel *ch, int num_states, int P, int L, uint64_t seed, uint8_t *codes) {
  if (num_states < 0 || P < 1 || L < 1 || L > 4) return 1;
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const int n = L * P;
  uint8_t *arrived = (uint8_t *)malloc((size_t)n);
  if (!arrived) return 2;
  for (int w = 0; w < num_states; ++w) {
    const or_channel c = ch[w];
    uint32_t out[4];
    uint32_t ctr[4] = {0xffffffffu, (uint32_t)w, OR_SAMPLER_TAG, 0u};
    or_philox4x32_10(ctr, key, out);
    int bad = (uint64_t)out[0] < or_threshold(c.p_start_bad);
    for (int s = 0; s < n; ++s) {
      const uint32_t cs[4] = {(uint32_t)(s >> 1), (uint32_t)w, OR_SAMPLER_TAG, 0u};
      or_philox4x32_10(cs, key, out);
      const uint32_t u_loss = (s & 1) ? out[2] : out[0];
      const uint32_t u_move = (s & 1) ? out[3] : out[1];
      int lost = (uint64_t)u_loss < or_threshold(bad ? c.loss_bad : c.loss_good);
      if (c.deadline >= 0 && s >= c.deadline) lost = 1;
      arrived[s] = (uint8_t)!lost;
      if (!bad) {
        if ((uint64_t)u_move < or_threshold(c.p_gb)) bad = 1;
      } else {
        if ((uint64_t)u_move < or_threshold(c.p_bg)) bad = 0;
      }
    }
    for (int p = 0; p < P; ++p) {
      int code = 0;
      while (code < L && arrived[code * P + p]) ++code;
      codes[(int64_t)w * P + p] = (uint8_t)code;
    }
  }
  free(arrived);
  return 0;
}
