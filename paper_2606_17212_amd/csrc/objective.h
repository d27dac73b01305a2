// Packet-conditioned rendering objective (Sec. 4, Eq. (2)) on the device:
// launch arguments and the scratch layout.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace dgs {

constexpr int kObjMaxImages = 65536;
constexpr int kObjMaxExpect = 4096;  // partial states ranked in LDS for the CVaR tail
constexpr int kObjMaxPairs = 65536;

struct ObjWeights {
  float lambda_ssim, lambda_c, alpha, lambda_t, lambda_m, lambda_a;
};

// Scratch sections (bytes from the start, 256-B aligned).
struct ObjLayout {
  size_t header;  // ObjHeader
  size_t dpart;   // double [K][blocks][2]: squared error and SSIM sums per 16x16 block
  size_t tpart;   // double [Q][blocks]: temporal squared error per block
  size_t maps;    // float [K][H][W][9]: SSIM gradient coefficients (a, b, c) per channel
  size_t cnt;     // int [5][K]: role counts (expect, tail, tail boundary, anchor, hinge sign)
  size_t coef;    // float [K]: dL/dD per image
  size_t tcnt;    // int [K + 1]: temporal pairs per image, then their offsets
  size_t tkey0, tkey1, tval0, tval1;  // u32 [2Q]: (image, (pair << 1) | later frame), sorted by image
  size_t thist;   // u32 radix histograms for 2Q keys
  size_t tparts;  // scan partials
  size_t d;       // float [K]: D per image
  size_t tsum;    // double [Q]: temporal squared error per pair
  size_t total;
};

struct ObjHeader {
  unsigned int bad;  // bit 0 index out of range, bit 1 list too long
};

ObjLayout make_obj_layout(int64_t K, int64_t width, int64_t height, int64_t Q);

struct ObjArgs {
  const float *images, *targets;
  const int32_t *target_of, *expect, *anchor, *mono, *temporal;
  int K, T, width, height, n_expect, n_anchor, n_mono, n_temporal;
  int bx, by;  // 16x16 blocks per row and column
  ObjWeights w;
  float *loss, *distortion, *grad;
  ObjHeader *hdr;
  double *dpart, *tpart, *tsum;
  float *maps, *coef, *d;
  int *cnt, *tcnt;
  uint32_t *tkey0, *tkey1, *tval0, *tval1, *thist;
  unsigned long long *tparts;
};

void launch_objective(const ObjArgs &a, hipStream_t st);

// Mean absolute error of images against their targets (the L1 training
// loss): scratch holds an ObjHeader, then one FP64 partial per
// (image, kL1Chunk elements).
constexpr int kL1Chunk = 4096;  // elements per workgroup (16 per thread)
size_t l1_scratch_bytes(int64_t K, int64_t width, int64_t height);
void launch_l1_loss(const float *images, int K, int64_t per_image, const float *targets, int T,
                    const int32_t *target_of, float *loss, void *scratch, hipStream_t st);
void launch_l1_grad(const float *images, int K, int64_t per_image, const float *targets, int T,
                    const int32_t *target_of, const float *dloss, float *grad, hipStream_t st);

}  // namespace dgs
