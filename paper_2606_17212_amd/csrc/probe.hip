// Measured roofs of the machine, next to the published peaks: a streaming
// copy (the HBM rate a plain read + write stream reaches) and two issue-rate
// probes, FP32 fused multiply-add and the hardware base-2 exponential, the
// two instruction kinds the compositing kernels are built from.
#include "../../include/dgs.h"
#include "common.h"

namespace dgs {

// dst[i] = src[i] for n float4 elements; grid-stride, 16-byte accesses.
__global__ void __launch_bounds__(kBlock) k_probe_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                        int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Eight independent dependency chains per lane, `iters` steps each.
// FMA: x = x * a + b (2 FLOPs per step and chain, |x| stays bounded since |a| < 1).
// EXP: x = 2^(-x) (one v_exp_f32 per step and chain; x stays in (0.5, 1)).
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_probe_valu(int64_t iters, float a, float b, float *__restrict__ out) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = 0.5f + 0.0625f * (float)k + 1e-7f * (float)(t & 63);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = KIND == 0 ? fmaf(x[k], a, b) : __builtin_amdgcn_exp2f(-x[k]);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[t] = s;
}

}  // namespace dgs

using namespace dgs;

extern "C" {

int dgs_probe_copy(const void *src, void *dst, size_t bytes, void *stream) {
  if (!src || !dst || bytes == 0 || (bytes & 15u) || (((uintptr_t)src | (uintptr_t)dst) & 15u)) return DGS_ERR_INVALID_ARG;
  const int64_t n = (int64_t)(bytes / 16);
  const int64_t blocks = ceil_div(n, kBlock) < 65536 ? ceil_div(n, kBlock) : 65536;
  k_probe_copy<<<(unsigned)blocks, kBlock, 0, (hipStream_t)stream>>>(static_cast<const float4 *>(src),
                                                                     static_cast<float4 *>(dst), n);
  return hipGetLastError() == hipSuccess ? DGS_OK : DGS_ERR_HIP;
}

int dgs_probe_valu(int32_t kind, int64_t iterations, float *out, void *stream) {
  if ((kind != 0 && kind != 1) || iterations < 1 || iterations > (1ll << 24) || !out) return DGS_ERR_INVALID_ARG;
  const unsigned blocks = DGS_PROBE_THREADS / kBlock;
  if (kind == 0)
    k_probe_valu<0><<<blocks, kBlock, 0, (hipStream_t)stream>>>(iterations, 0.999f, 0.001f, out);
  else
    k_probe_valu<1><<<blocks, kBlock, 0, (hipStream_t)stream>>>(iterations, 0.0f, 0.0f, out);
  return hipGetLastError() == hipSuccess ? DGS_OK : DGS_ERR_HIP;
}

}  // extern "C"
