// Per-Gaussian deformation (Eq. (1) of Sec. 3) and EWA projection, forward
// and backward.  One thread per Gaussian (or per Gaussian and delivered
// depth when the scene carries refinement levels), component-major (SoA)
// loads: lanes of a wave read consecutive floats of every component row, so
// each row is one coalesced stream.
//
// Refinement levels (Sec. 3: scale, rotation, opacity and colour are a base
// plus three refinements; the position has residual levels on top of the
// deformation): at delivered depth d an attribute is base + level 1 + ... +
// level d, each sum rounded once in that order; the position residual is
// summed the same way from zero and added to the deformed mean.
//
// The forward follows a fixed FP32 operation order (every product, quotient,
// square root and sum rounded once, no contraction; e^x by Cody-Waite
// reduction and a degree-7 Taylor polynomial).  Depth keys, culling and
// tile rectangles are therefore reproducible bit for bit by any implementation
// that takes the same steps.
#include "common.h"
#include "kernels.h"

namespace dgs {

// e^x: n = rint(x log2 e), r = (x - n ln2_hi) - n ln2_lo (Cody & Waite 1980),
// e^r from the Taylor polynomial of degree 7 in Horner form, scaled by 2^n.
__device__ inline float exp_cw(float x) {
  const float log2e = 0x1.715476p+0f;
  const float ln2_hi = 0x1.62e4p-1f;
  const float ln2_lo = 0x1.7f7d1cp-20f;
  float n = rintf(x * log2e);
  float r = (x - n * ln2_hi) - n * ln2_lo;
  float p = 0x1.a01a02p-13f;
  p = p * r + 0x1.6c16c2p-10f;
  p = p * r + 0x1.111112p-7f;
  p = p * r + 0x1.555556p-5f;
  p = p * r + 0x1.555556p-3f;
  p = p * r + 0.5f;
  p = p * r + 1.0f;
  p = p * r + 1.0f;
  return ldexpf(p, (int)n);
}

__device__ inline float clampf(float x, float lo, float hi) { return fminf(fmaxf(x, lo), hi); }

// Row `row` of Gaussian i's refinement levels 1..d added to x.
__device__ inline float refined(const SceneArgs &s, float x, int row, int64_t i, int d) {
  for (int j = 0; j < d; ++j) x = x + s.refine[((int64_t)j * s.refine_rows + row) * s.n + i];
  return x;
}

// Intermediate quantities of one Gaussian's projection.
struct Proj {
  float mu[3];
  float X, Y, Z, xz, yz, txz, tyz;
  float j00, j02, j11, j12;
  float qw, qx, qy, qz, qnorm;   // normalised quaternion and the raw norm
  float Rq[9];
  float vs[3];                   // e^{2 s_k}
  float M[6], V[6];
  float a, b, c, det, A, B, C;
  float u, v;
};

// d: delivered depth of a refined scene (0 and unused otherwise).
__device__ inline void project(const SceneArgs &s, const CamArgs &cam, int i, int d, Proj &p) {
  const int64_t n = s.n;
  const float m0 = s.mean[i], m1 = s.mean[n + i], m2 = s.mean[2 * n + i];
  int cl = 0;
  if (s.affine) {
    const int pk = (int)(s.packet_layer[i] >> 2);
    cl = (pk < s.num_packets ? pk : 0) / s.num_contexts;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float mk;
    if (s.affine) {
      const float *A = s.affine + 12 * cl + 4 * k;
      mk = ((A[0] * m0 + A[1] * m1) + A[2] * m2) + A[3];
    } else {
      mk = (k == 0) ? m0 : (k == 1) ? m1 : m2;
    }
    for (int r = 0; r < s.rank; ++r) mk = mk + s.basis[r] * s.temporal[(3 * r + k) * n + i];
    if (s.refine) mk = mk + refined(s, 0.0f, k, i, d);
    p.mu[k] = mk;
  }
  float P[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    P[k] = ((cam.R[3 * k] * p.mu[0] + cam.R[3 * k + 1] * p.mu[1]) + cam.R[3 * k + 2] * p.mu[2]) + cam.t[k];
  p.X = P[0]; p.Y = P[1]; p.Z = P[2];
  p.xz = p.X / p.Z;
  p.yz = p.Y / p.Z;
  p.u = cam.fx * p.xz + cam.cx;
  p.v = cam.fy * p.yz + cam.cy;
  const float limx = (0.65f * (float)cam.width) / cam.fx;
  const float limy = (0.65f * (float)cam.height) / cam.fy;
  p.txz = clampf(p.xz, -limx, limx);
  p.tyz = clampf(p.yz, -limy, limy);
  p.j00 = cam.fx / p.Z;
  p.j02 = -(cam.fx * p.txz) / p.Z;
  p.j11 = cam.fy / p.Z;
  p.j12 = -(cam.fy * p.tyz) / p.Z;

  const float qw = refined(s, s.quat[i], 6, i, d), qx = refined(s, s.quat[n + i], 7, i, d);
  const float qy = refined(s, s.quat[2 * n + i], 8, i, d), qz = refined(s, s.quat[3 * n + i], 9, i, d);
  const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  p.qnorm = sqrtf(n2);
  const float w = qw / p.qnorm, x = qx / p.qnorm, y = qy / p.qnorm, z = qz / p.qnorm;
  p.qw = w; p.qx = x; p.qy = y; p.qz = z;
  p.Rq[0] = 1.0f - 2.0f * (y * y + z * z);
  p.Rq[1] = 2.0f * (x * y - w * z);
  p.Rq[2] = 2.0f * (x * z + w * y);
  p.Rq[3] = 2.0f * (x * y + w * z);
  p.Rq[4] = 1.0f - 2.0f * (x * x + z * z);
  p.Rq[5] = 2.0f * (y * z - w * x);
  p.Rq[6] = 2.0f * (x * z - w * y);
  p.Rq[7] = 2.0f * (y * z + w * x);
  p.Rq[8] = 1.0f - 2.0f * (x * x + y * y);
#pragma unroll
  for (int k = 0; k < 3; ++k) p.vs[k] = exp_cw(2.0f * refined(s, s.log_scale[k * n + i], 3 + k, i, d));
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    p.M[j] = p.j00 * cam.R[j] + p.j02 * cam.R[6 + j];
    p.M[3 + j] = p.j11 * cam.R[3 + j] + p.j12 * cam.R[6 + j];
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      p.V[3 * r + j] = (p.M[3 * r] * p.Rq[j] + p.M[3 * r + 1] * p.Rq[3 + j]) + p.M[3 * r + 2] * p.Rq[6 + j];
  const float *V = p.V;
  p.a = (((V[0] * V[0]) * p.vs[0] + (V[1] * V[1]) * p.vs[1]) + (V[2] * V[2]) * p.vs[2]) + kDilation;
  p.b = ((V[0] * V[3]) * p.vs[0] + (V[1] * V[4]) * p.vs[1]) + (V[2] * V[5]) * p.vs[2];
  p.c = (((V[3] * V[3]) * p.vs[0] + (V[4] * V[4]) * p.vs[1]) + (V[5] * V[5]) * p.vs[2]) + kDilation;
  p.det = p.a * p.c - p.b * p.b;
  p.A = p.c / p.det;
  p.B = -p.b / p.det;
  p.C = p.a / p.det;
}

// Colour: RGB, or degree-1 real SH (Condon-Shortley phase) + 0.5 clamped at 0
// along the direction from the camera centre to the deformed mean.
__device__ inline void colour(const SceneArgs &s, const CamArgs &cam, int i, int d, const float mu[3],
                              float col[3], float dir[3], float raw[3]) {
  const int64_t n = s.n;
  if (s.sh_degree == 0) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) { col[ch] = refined(s, s.color[ch * n + i], 11 + ch, i, d); raw[ch] = col[ch]; }
    dir[0] = dir[1] = dir[2] = 0.0f;
    return;
  }
  float d0 = mu[0] - cam.campos[0], d1 = mu[1] - cam.campos[1], d2 = mu[2] - cam.campos[2];
  float inv = 1.0f / sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
  dir[0] = d0 * inv; dir[1] = d1 * inv; dir[2] = d2 * inv;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    const float k0 = refined(s, s.color[ch * n + i], 11 + ch, i, d);
    const float k1 = refined(s, s.color[(3 + ch) * n + i], 14 + ch, i, d);
    const float k2 = refined(s, s.color[(6 + ch) * n + i], 17 + ch, i, d);
    const float k3 = refined(s, s.color[(9 + ch) * n + i], 20 + ch, i, d);
    float val = 0.5f + kShC0 * k0 + kShC1 * (-dir[1] * k1 + dir[2] * k2 - dir[0] * k3);
    raw[ch] = val;
    col[ch] = fmaxf(val, 0.0f);
  }
}

// REFINED: one thread per record slot v = 4 i + d (Gaussian i at delivered
// depth d); the slot exists when d >= the Gaussian's layer, and its record
// carries (packet << 2) | d so that the compositing tables select it in the
// states that deliver exactly depth d.
template <bool REFINED>
__global__ void __launch_bounds__(kBlock)
k_geometry(SceneArgs s, CamArgs cam, TileArgs tl, const uint32_t *__restrict__ list,
           const unsigned *__restrict__ n_active, float4 *__restrict__ rec0,
           float4 *__restrict__ rec1, float4 *__restrict__ rec2, uint2 *__restrict__ rect,
           uint2 *__restrict__ pbox, uint4 *__restrict__ brec, uint32_t *__restrict__ dkey,
           uint32_t *__restrict__ dval, uint32_t *__restrict__ plhist) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  const int nact = list ? (int)*n_active : (REFINED ? 4 * s.n : s.n);
  if (j >= nact) return;
  const int v = list ? (int)list[j] : j;
  const int i = REFINED ? (v >> 2) : v;
  const int d = REFINED ? (v & 3) : 0;
  if (plhist && d == 0) {  // Gaussians per (packet, layer): each Gaussian once
    const int pl0 = s.packet_layer[i];
    if (pl0 < 4 * s.num_packets) atomicAdd(plhist + (pl0 >> 2) * kPlStride + (pl0 & 3), 1u);
  }
  Proj p;
  project(s, cam, i, d, p);
  float col[3], dir[3], raw[3];
  colour(s, cam, i, d, p.mu, col, dir, raw);
  // log2 of the opacity: alpha = min(0.99, 2^(q' + log2 o)) in the compositing kernels
  const float lo = -__log2f(1.0f + __expf(-refined(s, s.opacity_logit[i], 10, i, d)));
  uint16_t pl = s.packet_layer[i];
  bool exists = true;
  if (REFINED) {
    exists = (int)(pl & 3u) <= d;
    pl = (uint16_t)((pl & ~3u) | (uint32_t)d);
  }
  // a packet id outside the state tables never enters a list
  const bool ok = exists && (p.Z > cam.near_z) && (p.det > 0.0f) && ((int)(pl >> 2) < s.num_packets);
  uint32_t x0 = 0, y0 = 0, x1 = 0, y1 = 0, px0 = 0, py0 = 0, px1 = 0, py1 = 0;
  if (ok) {
    const float itw = 1.0f / (float)tl.tile_w, ith = 1.0f / (float)tl.tile_h;
    const float ex = sqrtf(kQCut * p.a), ey = sqrtf(kQCut * p.c);
    x0 = (uint32_t)clampf(floorf((p.u - ex) * itw), 0.0f, (float)tl.tiles_x);
    x1 = (uint32_t)clampf(floorf((p.u + ex) * itw) + 1.0f, 0.0f, (float)tl.tiles_x);
    y0 = (uint32_t)clampf(floorf((p.v - ey) * ith), 0.0f, (float)tl.tiles_y);
    y1 = (uint32_t)clampf(floorf((p.v + ey) * ith) + 1.0f, 0.0f, (float)tl.tiles_y);
    // the same rectangle in pixels (half-open): a pixel centre outside it has alpha < 1/255
    px0 = (uint32_t)clampf(floorf(p.u - ex), 0.0f, (float)cam.width);
    px1 = (uint32_t)clampf(floorf(p.u + ex) + 1.0f, 0.0f, (float)cam.width);
    py0 = (uint32_t)clampf(floorf(p.v - ey), 0.0f, (float)cam.height);
    py1 = (uint32_t)clampf(floorf(p.v + ey) + 1.0f, 0.0f, (float)cam.height);
  }
  // conic pre-scaled so that q' = A' dx^2 + B' dx dy + C' dy^2 = -(q/2) log2 e
  const float cA = kConicA * p.A, cB = kConicB * p.B, cC = kConicA * p.C;
  const uint2 rt = make_uint2(x0 | (y0 << 16), x1 | (y1 << 16));
  rec0[v] = make_float4(p.u, p.v, lo, __uint_as_float((uint32_t)pl));
  rec1[v] = make_float4(cA, cB, cC, p.Z);
  rec2[v] = make_float4(col[0], col[1], col[2], 0.0f);
  rect[v] = rt;
  pbox[v] = make_uint2(px0 | (py0 << 16), px1 | (py1 << 16));
  // what the level-2 instance scatter reads per list entry, in one 32-byte
  // record: the rectangle, the centre, the conic and the exponent bound of
  // the reach ellipse, q' >= log2(1/255) - 0.01 - log2 o
  brec[2 * (int64_t)v] = make_uint4(rt.x, rt.y, __float_as_uint(p.u), __float_as_uint(p.v));
  brec[2 * (int64_t)v + 1] = make_uint4(__float_as_uint(cA), __float_as_uint(cB), __float_as_uint(cC),
                                        __float_as_uint(kQSkip - 0.01f - lo));
  const bool nonempty = ok && x1 > x0 && y1 > y0;
  dkey[j] = nonempty ? __float_as_uint(p.Z) : 0xFFFFFFFFu;
  dval[j] = (uint32_t)v;
}

// Gradients of one projected record with respect to the attributes it was
// projected from: the deformed mean, log-scale, raw quaternion, opacity logit
// and colour coefficients (at the record's delivered depth d with refinement
// levels).  Discrete decisions are frozen: the clamps of x/z, y/z and of the
// SH colour pass zero gradient; depth only orders and carries none.
struct AttrGrad {
  float mu[3], ls[3], q[4], logit, col[12];
};

__device__ inline void zero_grad(AttrGrad &g) {
#pragma unroll
  for (int k = 0; k < 3; ++k) g.mu[k] = g.ls[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) g.q[k] = 0.0f;
  g.logit = 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) g.col[k] = 0.0f;
}

__device__ inline void add_grad(AttrGrad &a, const AttrGrad &b) {
#pragma unroll
  for (int k = 0; k < 3; ++k) { a.mu[k] += b.mu[k]; a.ls[k] += b.ls[k]; }
#pragma unroll
  for (int k = 0; k < 4; ++k) a.q[k] += b.q[k];
  a.logit += b.logit;
#pragma unroll
  for (int k = 0; k < 12; ++k) a.col[k] += b.col[k];
}

// g2d: [9][nrec] gradients of record v w.r.t. (u, v, A', B', C', log2 o, r, g, b).
// Returns false (and leaves g zero) for a record that received no gradient.
__device__ inline bool record_grads(const SceneArgs &s, const CamArgs &cam, const float *__restrict__ g2d,
                                    int64_t nrec, int64_t v, int i, int d, AttrGrad &g) {
  zero_grad(g);
  // the compositing backward differentiates w.r.t. (u, v, A', B', C', log2 o): undo the scalings
  const float gu = g2d[v], gv = g2d[nrec + v];
  const float gA = kConicA * g2d[2 * nrec + v], gB = kConicB * g2d[3 * nrec + v];
  const float gC = kConicA * g2d[4 * nrec + v], glo = g2d[5 * nrec + v];
  const float gcol[3] = {g2d[6 * nrec + v], g2d[7 * nrec + v], g2d[8 * nrec + v]};
  if (gu == 0.0f && gv == 0.0f && gA == 0.0f && gB == 0.0f && gC == 0.0f && glo == 0.0f && gcol[0] == 0.0f &&
      gcol[1] == 0.0f && gcol[2] == 0.0f)
    return false;  // not composited anywhere (or culled): nothing flows back
  const int64_t n = s.n;
  Proj p;
  project(s, cam, i, d, p);
  float col[3], dir[3], raw[3];
  colour(s, cam, i, d, p.mu, col, dir, raw);

  // opacity: log2 o = -log2(1 + e^{-logit}), d/dlogit = (1 - o) / ln 2
  const float o = 1.0f / (1.0f + __expf(-refined(s, s.opacity_logit[i], 10, i, d)));
  g.logit = glo * (1.0f - o) * 1.4426950408889634f;

  // colour
  if (s.sh_degree == 0) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) g.col[ch] = gcol[ch];
  } else {
    float gd[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float gr = raw[ch] > 0.0f ? gcol[ch] : 0.0f;
      const float k1 = refined(s, s.color[(3 + ch) * n + i], 14 + ch, i, d);
      const float k2 = refined(s, s.color[(6 + ch) * n + i], 17 + ch, i, d);
      const float k3 = refined(s, s.color[(9 + ch) * n + i], 20 + ch, i, d);
      g.col[ch] = kShC0 * gr;
      g.col[3 + ch] = -kShC1 * dir[1] * gr;
      g.col[6 + ch] = kShC1 * dir[2] * gr;
      g.col[9 + ch] = -kShC1 * dir[0] * gr;
      gd[0] += -kShC1 * k3 * gr;
      gd[1] += -kShC1 * k1 * gr;
      gd[2] += kShC1 * k2 * gr;
    }
    const float e0 = p.mu[0] - cam.campos[0], e1 = p.mu[1] - cam.campos[1], e2 = p.mu[2] - cam.campos[2];
    const float inv = 1.0f / sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
    const float dd = dir[0] * gd[0] + dir[1] * gd[1] + dir[2] * gd[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) g.mu[k] += (gd[k] - dir[k] * dd) * inv;
  }

  // conic (A, B, C) -> 2D covariance (a, b, c): d(Sigma^-1) = -Sigma^-1 dSigma Sigma^-1
  const float A = p.A, B = p.B, C = p.C;
  const float ga = -(A * A * gA + A * B * gB + B * B * gC);
  const float gb = -(2.0f * A * B * gA + (A * C + B * B) * gB + 2.0f * B * C * gC);
  const float gc = -(B * B * gA + B * C * gB + C * C * gC);

  // (a, b, c) -> V (2x3) and the scale variances
  float gV[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float v0 = p.V[k], v1 = p.V[3 + k], vs = p.vs[k];
    gV[k] = (2.0f * ga * v0 + gb * v1) * vs;
    gV[3 + k] = (2.0f * gc * v1 + gb * v0) * vs;
    const float gvs = ga * v0 * v0 + gb * v0 * v1 + gc * v1 * v1;
    g.ls[k] = 2.0f * vs * gvs;
  }

  // V = M Rq
  float gM[6], gR[9];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      gM[3 * r + j] = gV[3 * r] * p.Rq[3 * j] + gV[3 * r + 1] * p.Rq[3 * j + 1] + gV[3 * r + 2] * p.Rq[3 * j + 2];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int l = 0; l < 3; ++l) gR[3 * j + l] = p.M[j] * gV[l] + p.M[3 + j] * gV[3 + l];

  // M = J R_cw
  float gj00 = 0.0f, gj02 = 0.0f, gj11 = 0.0f, gj12 = 0.0f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    gj00 += gM[j] * cam.R[j];
    gj02 += gM[j] * cam.R[6 + j];
    gj11 += gM[3 + j] * cam.R[3 + j];
    gj12 += gM[3 + j] * cam.R[6 + j];
  }
  // J and (u, v) -> camera-frame mean
  const float iz = 1.0f / p.Z, iz2 = iz * iz;
  const float fx = cam.fx, fy = cam.fy;
  const bool inx = p.txz == p.xz, iny = p.tyz == p.yz;
  float gX = gu * fx * iz + (inx ? -gj02 * fx * iz2 : 0.0f);
  float gY = gv * fy * iz + (iny ? -gj12 * fy * iz2 : 0.0f);
  float gZ = -gu * fx * p.xz * iz - gv * fy * p.yz * iz - gj00 * fx * iz2 - gj11 * fy * iz2 +
             gj02 * fx * (inx ? 2.0f * p.xz : p.txz) * iz2 +
             gj12 * fy * (iny ? 2.0f * p.yz : p.tyz) * iz2;
  // P = R_cw mu + t
#pragma unroll
  for (int k = 0; k < 3; ++k) g.mu[k] += cam.R[k] * gX + cam.R[3 + k] * gY + cam.R[6 + k] * gZ;

  // rotation -> normalised quaternion -> raw quaternion
  const float w = p.qw, x = p.qx, y = p.qy, z = p.qz;
  const float gw = 2.0f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
  const float gx = 2.0f * (y * gR[1] + z * gR[2] + y * gR[3] - 2.0f * x * gR[4] - w * gR[5] +
                           z * gR[6] + w * gR[7] - 2.0f * x * gR[8]);
  const float gy = 2.0f * (-2.0f * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] -
                           w * gR[6] + z * gR[7] - 2.0f * y * gR[8]);
  const float gz = 2.0f * (-2.0f * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0f * z * gR[4] +
                           y * gR[5] + x * gR[6] + y * gR[7]);
  const float dq = w * gw + x * gx + y * gy + z * gz;
  const float iq = 1.0f / p.qnorm;
  g.q[0] = (gw - w * dq) * iq;
  g.q[1] = (gx - x * dq) * iq;
  g.q[2] = (gy - y * dq) * iq;
  g.q[3] = (gz - z * dq) * iq;
  return true;
}

// Base parameter gradients from attribute gradients: the deformation
// mu = A_c [m; 1] + sum_r b_r q_r takes the mean's share.
__device__ inline void write_base_grads(const SceneArgs &s, int64_t i, const AttrGrad &g, float *__restrict__ g_mean,
                                        float *__restrict__ g_ls, float *__restrict__ g_quat,
                                        float *__restrict__ g_logit, float *__restrict__ g_color,
                                        float *__restrict__ g_temporal) {
  const int64_t n = s.n;
  g_logit[i] = g.logit;
  const int ncol = s.sh_degree == 0 ? 3 : 12;
  for (int k = 0; k < ncol; ++k) g_color[k * n + i] = g.col[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) g_ls[k * n + i] = g.ls[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) g_quat[k * n + i] = g.q[k];
  if (s.affine) {
    const int pk = (int)(s.packet_layer[i] >> 2);
    const int cl = (pk < s.num_packets ? pk : 0) / s.num_contexts;
    const float *Af = s.affine + 12 * cl;
#pragma unroll
    for (int j = 0; j < 3; ++j) g_mean[j * n + i] = Af[j] * g.mu[0] + Af[4 + j] * g.mu[1] + Af[8 + j] * g.mu[2];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) g_mean[k * n + i] = g.mu[k];
  }
  for (int r = 0; r < s.rank; ++r)
#pragma unroll
    for (int k = 0; k < 3; ++k) g_temporal[(3 * r + k) * n + i] = s.basis[r] * g.mu[k];
}

// REFINED: one thread per Gaussian walks its records from depth 3 down; the
// running sum over depths >= d is the gradient of level d (every record of
// depth >= d carries level d), the full sum the base parameters'.  g_refine:
// [3][rows][n] in the layout of the scene's levels.
template <bool REFINED>
__global__ void __launch_bounds__(kBlock)
k_geometry_bwd(SceneArgs s, CamArgs cam, const float *__restrict__ g2d, float *__restrict__ g_mean,
               float *__restrict__ g_ls, float *__restrict__ g_quat, float *__restrict__ g_logit,
               float *__restrict__ g_color, float *__restrict__ g_temporal, float *__restrict__ g_refine) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int64_t n = s.n;
  if (i >= n) return;
  AttrGrad acc;
  if (!REFINED) {
    record_grads(s, cam, g2d, n, i, i, 0, acc);
  } else {
    zero_grad(acc);
    const int layer = (int)(s.packet_layer[i] & 3u);
    const int ncol = s.sh_degree == 0 ? 3 : 12;
    const int64_t rows = s.refine_rows;
#pragma unroll 1
    for (int d = 3; d >= 0; --d) {
      AttrGrad g;
      if (d >= layer && record_grads(s, cam, g2d, 4 * n, 4 * (int64_t)i + d, i, d, g)) add_grad(acc, g);
      if (d >= 1) {
        float *L = g_refine + (int64_t)(d - 1) * rows * n + i;
#pragma unroll
        for (int k = 0; k < 3; ++k) L[k * n] = acc.mu[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) L[(3 + k) * n] = acc.ls[k];
#pragma unroll
        for (int k = 0; k < 4; ++k) L[(6 + k) * n] = acc.q[k];
        L[10 * n] = acc.logit;
        for (int k = 0; k < ncol; ++k) L[(11 + k) * n] = acc.col[k];
      }
    }
  }
  write_base_grads(s, i, acc, g_mean, g_ls, g_quat, g_logit, g_color, g_temporal);
}

// ------------------------------------------------------------------ launchers

void launch_geometry(const SceneArgs &s, const CamArgs &c, const TileArgs &t, const uint32_t *list,
                     const unsigned *n_active, int grid_n, float4 *rec0, float4 *rec1, float4 *rec2,
                     uint2 *rect, uint2 *pbox, uint4 *brec, uint32_t *dkey, uint32_t *dval, hipStream_t st,
                     uint32_t *plhist) {
  if (grid_n <= 0) return;
  if (list) plhist = nullptr;  // a list covers a subset: the histogram needs every Gaussian
  if (s.refine)
    k_geometry<true><<<(unsigned)ceil_div(grid_n, kBlock), kBlock, 0, st>>>(s, c, t, list, n_active, rec0, rec1,
                                                                            rec2, rect, pbox, brec, dkey, dval, plhist);
  else
    k_geometry<false><<<(unsigned)ceil_div(grid_n, kBlock), kBlock, 0, st>>>(s, c, t, list, n_active, rec0, rec1,
                                                                             rec2, rect, pbox, brec, dkey, dval, plhist);
}

void launch_geometry_bwd(const SceneArgs &s, const CamArgs &c, const float *g2d, float *g_mean,
                         float *g_ls, float *g_quat, float *g_logit, float *g_color, float *g_temporal,
                         float *g_refine, hipStream_t st) {
  if (s.n <= 0) return;
  if (s.refine)
    k_geometry_bwd<true><<<(unsigned)ceil_div(s.n, kBlock), kBlock, 0, st>>>(s, c, g2d, g_mean, g_ls, g_quat,
                                                                             g_logit, g_color, g_temporal, g_refine);
  else
    k_geometry_bwd<false><<<(unsigned)ceil_div(s.n, kBlock), kBlock, 0, st>>>(s, c, g2d, g_mean, g_ls, g_quat,
                                                                              g_logit, g_color, g_temporal, nullptr);
}

}  // namespace dgs
