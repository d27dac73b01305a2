// Device-wide exclusive scan and stable LSD radix sort of (u32 key, u32 value)
// pairs, written for wave64.
//
// Both are reduce-then-scan: a reduction pass, a single-workgroup scan of the
// per-workgroup partials, and a pass that scans each workgroup's chunk with
// its offset.  No workgroup waits on another, so nothing depends on the order
// or concurrency in which workgroups are dispatched.
//
// Radix ranking inside a workgroup: each wave owns a contiguous run of
// 64 x IPT keys (IPT = 4, 8 or 16 keys per lane, smaller for smaller sorts so
// that more workgroups share a pass) and takes them 64 at a time; lanes
// holding the same digit find each other with one ballot per digit bit, the
// lane count below gives the rank
// within the round, and a per-(wave, digit) counter in LDS carries the rank
// across rounds.  No LDS atomics, so heavily skewed digits (the high bytes of
// depth keys) cost the same as uniform ones.  Keys are then scattered to LDS
// in block-sorted order and written out so that consecutive lanes write
// consecutive addresses of the same digit bucket.
#include "common.h"
#include "kernels.h"

namespace dgs {

// ------------------------------------------------------------------- scan

__global__ void __launch_bounds__(kBlock)
k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, unsigned long long *__restrict__ parts) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int64_t idx = base + k * kBlock + threadIdx.x;
    if (idx < n) s += in[idx];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, kWave);
  __shared__ unsigned long long ws[4];
  if (__lane_id() == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) parts[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// Exclusive scan of parts[0..np) in place by one 1024-thread workgroup.
__global__ void __launch_bounds__(1024)
k_scan_parts(unsigned long long *__restrict__ parts, int64_t np, unsigned long long *__restrict__ total) {
  __shared__ unsigned long long wsum[16];
  __shared__ unsigned long long carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  for (int64_t c0 = 0; c0 < np; c0 += 1024) {
    const int64_t idx = c0 + threadIdx.x;
    const unsigned long long x = idx < np ? parts[idx] : 0ull;
    const unsigned long long incl = wave_incl_scan(x);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    unsigned long long off = carry_s;
    for (int k = 0; k < w; ++k) off += wsum[k];
    if (idx < np) parts[idx] = off + incl - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry_s = off + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry_s;
}

__global__ void __launch_bounds__(kBlock)
k_scan_down(const uint32_t *in, uint32_t *out, int64_t n, const unsigned long long *__restrict__ parts) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const int64_t wbase = (int64_t)blockIdx.x * kScanTile + w * 1024;
  uint32_t v[16];
  uint32_t tot = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t idx = wbase + r * kWave + lane;
    v[r] = idx < n ? in[idx] : 0u;
    tot += v[r];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, kWave);
  __shared__ unsigned long long wsum[4];
  if (lane == 0) wsum[w] = tot;
  __syncthreads();
  unsigned long long carry = parts[blockIdx.x];
  for (int k = 0; k < w; ++k) carry += wsum[k];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint32_t incl = wave_incl_scan(v[r]);
    const int64_t idx = wbase + r * kWave + lane;
    if (idx < n) out[idx] = (uint32_t)(carry + incl - v[r]);
    carry += (uint32_t)__shfl(incl, 63, kWave);
  }
}

void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, unsigned long long *parts,
                     unsigned long long *total, hipStream_t st) {
  const int64_t nb = n > 0 ? ceil_div(n, kScanTile) : 1;
  k_scan_reduce<<<(unsigned)nb, kBlock, 0, st>>>(in, n, parts);
  k_scan_parts<<<1, 1024, 0, st>>>(parts, nb, total);
  if (n > 0) k_scan_down<<<(unsigned)nb, kBlock, 0, st>>>(in, out, n, parts);
}

// -------------------------------------------------------------- radix sort

__device__ inline int64_t sort_count(const void *count_dev, int is_u64, int64_t max_count) {
  if (!count_dev) return max_count;
  const int64_t c = is_u64 ? (int64_t)(*(const unsigned long long *)count_dev)
                           : (int64_t)(*(const unsigned *)count_dev);
  return c < max_count ? c : max_count;
}

// Digit of `key` for this pass, the mask of the lanes of this wave holding the
// same digit (among `active` lanes), found with one ballot per digit bit.
__device__ inline unsigned long long match_digit(uint32_t d, int nbits, unsigned long long active) {
  unsigned long long peers = active;
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const unsigned long long bb = __ballot(bit);
    peers &= bit ? bb : ~bb;
  }
  return peers;
}

// Per-block digit counts: digit-major (hist[d * nblocks + b], the order a
// flat scan turns into global offsets) or, for the scatter that forms its
// offsets itself, block-major (hist[b * 256 + d]: each block's counts one
// contiguous row, so that the scatter's walk over the blocks reads whole
// lines).
template <int IPT>
__global__ void __launch_bounds__(kBlock)
k_radix_up(const uint32_t *__restrict__ keys, const void *count_dev, int is_u64, int64_t max_count,
           int shift, int nbits, uint32_t *__restrict__ hist, int nblocks, int block_major) {
  __shared__ uint32_t wc[4][256];
  const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  wc[0][tid] = 0; wc[1][tid] = 0; wc[2][tid] = 0; wc[3][tid] = 0;
  __syncthreads();
  const int64_t n = sort_count(count_dev, is_u64, max_count);
  const uint32_t mask = (1u << nbits) - 1u;
  const int64_t wbase = (int64_t)blockIdx.x * (kBlock * IPT) + w * (kWave * IPT);
  if (wbase < n) {
    // all of the lane's loads in flight before the first digit is ranked
    uint32_t key[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const int64_t idx = wbase + r * kWave + lane;
      key[r] = idx < n ? keys[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const bool valid = wbase + r * kWave + lane < n;
      const uint32_t d = valid ? (key[r] >> shift) & mask : 0u;
      const unsigned long long peers = match_digit(d, nbits, __ballot(valid));
      if (valid && (peers & lanemask_gt()) == 0ull) wc[w][d] += (uint32_t)__popcll(peers);
    }
  }
  __syncthreads();
  if (tid <= (int)mask) {
    const int64_t at = block_major ? (int64_t)blockIdx.x * 256 + tid : (int64_t)tid * nblocks + blockIdx.x;
    hist[at] = wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
  }
}

template <int IPT>
__global__ void __launch_bounds__(kBlock)
k_radix_down(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
             uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, const void *count_dev,
             int is_u64, int64_t max_count, int shift, int nbits, const uint32_t *__restrict__ hist,
             int nblocks, int fused) {
  constexpr int kTile = kBlock * IPT;
  __shared__ uint32_t wc[4][256];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t skey[kTile];
  __shared__ uint32_t sval[kTile];
  const int64_t n = sort_count(count_dev, is_u64, max_count);
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (base >= n) return;  // uniform over the workgroup
  const int tid = threadIdx.x, lane = __lane_id(), w = tid >> 6;
  const uint32_t mask = (1u << nbits) - 1u;
  if (fused) {
    // global offset of (digit d, this block) from the raw block-major
    // histograms: sum over all blocks of the lower digits + this digit in
    // earlier blocks (the lanes of a wave read consecutive words of a row).
    // Done first, while the keys do not hold registers yet, so that many of
    // these loads are in flight at once.
    const int d = tid;
    uint32_t tot = 0, before = 0;
    if (d <= (int)mask) {
#pragma unroll 16
      for (int b = 0; b < nblocks; ++b) {
        const uint32_t c = hist[(int64_t)b * 256 + d];
        tot += c;
        before += b < (int)blockIdx.x ? c : 0u;
      }
    }
    const uint32_t incl = wave_incl_scan(tot);
    __syncthreads();
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += wsum[k];
    gbase[d] = off + incl - tot + before;
  }
  wc[0][tid] = 0; wc[1][tid] = 0; wc[2][tid] = 0; wc[3][tid] = 0;
  __syncthreads();
  uint32_t key[IPT], val[IPT], rank[IPT];
  const int64_t wbase = base + w * (kWave * IPT);
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int64_t idx = wbase + r * kWave + lane;
    key[r] = idx < n ? kin[idx] : 0u;
    val[r] = idx < n ? vin[idx] : 0u;
  }
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const bool valid = wbase + r * kWave + lane < n;
    const uint32_t d = (key[r] >> shift) & mask;
    const unsigned long long peers = match_digit(d, nbits, __ballot(valid));
    const uint32_t before = wc[w][d];
    rank[r] = before + (uint32_t)__popcll(peers & lanemask_lt());
    if (valid && (peers & lanemask_gt()) == 0ull) wc[w][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    const int d = tid;
    const uint32_t c0 = wc[0][d], c1 = wc[1][d], c2 = wc[2][d], c3 = wc[3][d];
    const uint32_t tot = c0 + c1 + c2 + c3;
    const uint32_t incl = wave_incl_scan(tot);
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += wsum[k];
    const uint32_t ex = off + incl - tot;
    dstart[d] = ex;
    wc[0][d] = ex;
    wc[1][d] = ex + c0;
    wc[2][d] = ex + c0 + c1;
    wc[3][d] = ex + c0 + c1 + c2;
    if (!fused) gbase[d] = (d <= (int)mask) ? hist[(int64_t)d * nblocks + blockIdx.x] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const int64_t idx = wbase + r * kWave + lane;
    if (idx < n) {
      const uint32_t d = (key[r] >> shift) & mask;
      const uint32_t pos = wc[w][d] + rank[r];
      skey[pos] = key[r];
      sval[pos] = val[r];
    }
  }
  __syncthreads();
  const int cnt = (int)((n - base) < kTile ? (n - base) : kTile);
  for (int k = tid; k < cnt; k += kBlock) {
    const uint32_t kk = skey[k];
    const uint32_t d = (kk >> shift) & mask;
    const uint32_t o = gbase[d] + (uint32_t)(k - (int)dstart[d]);
    if (kout) kout[o] = kk;
    vout[o] = sval[k];
  }
}

constexpr int kFusedScanBlocks = 256;

int launch_radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, const void *count_dev,
                      int count_is_u64, int64_t max_count, int begin_bit, int end_bit, uint32_t *hist,
                      unsigned long long *parts, hipStream_t st, bool last_pass_keys) {
  if (max_count <= 0) return 0;
  const int tile = sort_tile_for(max_count);
  const int nblocks = (int)ceil_div(max_count, tile);
  // fewest passes of <= 8 bits, digits as equal as possible (13 bits -> 7 + 6):
  // fewer buckets per pass give longer contiguous runs in the scatter
  const int total_bits = end_bit - begin_bit;
  const int passes = (total_bits + 7) / 8;
  int cur = 0;
  for (int pass = 0, shift = begin_bit; pass < passes; ++pass) {
    const int nbits = (total_bits - (shift - begin_bit) + (passes - pass) - 1) / (passes - pass);
    uint32_t *ki = cur ? k1 : k0, *vi = cur ? v1 : v0;
    uint32_t *ko = cur ? k0 : k1, *vo = cur ? v0 : v1;
    // few blocks: each scatter workgroup forms its digit offsets from the raw
    // histograms itself (no separate scan launches)
    const int fused = nblocks <= kFusedScanBlocks ? 1 : 0;
    if (tile == 1024)
      k_radix_up<4><<<nblocks, kBlock, 0, st>>>(ki, count_dev, count_is_u64, max_count, shift, nbits, hist, nblocks,
                                                fused);
    else if (tile == 2048)
      k_radix_up<8><<<nblocks, kBlock, 0, st>>>(ki, count_dev, count_is_u64, max_count, shift, nbits, hist, nblocks,
                                                fused);
    else
      k_radix_up<16><<<nblocks, kBlock, 0, st>>>(ki, count_dev, count_is_u64, max_count, shift, nbits, hist,
                                                 nblocks, fused);
    if (!fused) launch_scan_u32(hist, hist, (int64_t)(1 << nbits) * nblocks, parts, nullptr, st);
    uint32_t *kwrite = (pass == passes - 1 && !last_pass_keys) ? nullptr : ko;
    if (tile == 1024)
      k_radix_down<4><<<nblocks, kBlock, 0, st>>>(ki, vi, kwrite, vo, count_dev, count_is_u64, max_count, shift,
                                                  nbits, hist, nblocks, fused);
    else if (tile == 2048)
      k_radix_down<8><<<nblocks, kBlock, 0, st>>>(ki, vi, kwrite, vo, count_dev, count_is_u64, max_count, shift,
                                                  nbits, hist, nblocks, fused);
    else
      k_radix_down<16><<<nblocks, kBlock, 0, st>>>(ki, vi, kwrite, vo, count_dev, count_is_u64, max_count, shift,
                                                   nbits, hist, nblocks, fused);
    cur ^= 1;
    shift += nbits;
  }
  return cur;
}

}  // namespace dgs
