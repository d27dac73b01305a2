// Delivery-state sampler (Sec. 4: training worlds sample erasures from an IID
// and a Gilbert-Elliott burst process; dependencies are enforced after
// delivery and become cluster-layer masks), on the device so that sweeps and
// captured graphs draw their states without host traffic.
//
// Every (packet p, layer l) is one datagram, sent layer-major: slot
// s = l P + p.  A world's channel is a two-state Markov chain over the slots:
// the datagram of slot s is erased with the current state's loss probability,
// then the chain moves (good -> bad with p_gb, bad -> good with p_bg); the
// first state is bad with probability p_start_bad.  Slots >= deadline arrive
// too late.  A packet's code is its number of leading arrived layers.
//
// Draws: Philox4x32-10 keyed by the seed; counter (s / 2, w, 0x44475331, 0)
// gives (erasure, transition) for slot s from outputs (0, 1) (even s) or
// (2, 3) (odd s); counter (0xffffffff, w, 0x44475331, 0) output 0 draws the
// first state.  An event of probability p happens when the 32-bit draw is
// below floor(p 2^32).
//
// One wave per world; lane i simulates a contiguous run of slots.  The chain
// does not depend on the erasures, so pass 1 runs each lane's slots from both
// possible start states, one thread chains the 64 runs, and pass 2 replays each
// run from its true start state, drawing the erasures into an LDS bitmap.

#include <math.h>

#include "common.h"
#include "kernels.h"

namespace dgs {

constexpr uint32_t kSamplerTag = 0x44475331u;

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t y0 = hi1 ^ c1 ^ k0, y2 = hi0 ^ c3 ^ k1;
    c0 = y0;
    c1 = lo1;
    c2 = y2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__device__ __forceinline__ uint64_t event_threshold(float p) {
  if (!(p > 0.0f)) return 0ull;
  if (p >= 1.0f) return 1ull << 32;
  return (uint64_t)floor((double)p * 4294967296.0);
}

// Draws of slot s of world w: (erasure, transition).
struct SlotDraws {
  uint32_t pair = 0xffffffffu;  // s / 2 of the cached Philox block
  uint32_t out[4];
  __device__ __forceinline__ void get(uint32_t s, uint32_t w, uint32_t k0, uint32_t k1, uint32_t &u_loss,
                                      uint32_t &u_move) {
    if ((s >> 1) != pair) {
      pair = s >> 1;
      philox4x32_10(pair, w, kSamplerTag, 0u, k0, k1, out);
    }
    u_loss = (s & 1u) ? out[2] : out[0];
    u_move = (s & 1u) ? out[3] : out[1];
  }
};

__global__ void __launch_bounds__(kWave)
k_sample_states(const SamplerChannel *__restrict__ ch, int P, int L, uint32_t k0, uint32_t k1,
                uint8_t *__restrict__ codes) {
  extern __shared__ uint32_t arrived[];  // ceil(L P / 32) words
  __shared__ uint32_t maps[kWave];       // bit 0: end state from good, bit 1: from bad
  __shared__ uint32_t starts[kWave];
  const uint32_t w = blockIdx.x;
  const int lane = threadIdx.x;
  const SamplerChannel c = ch[w];
  const uint64_t t_gb = event_threshold(c.p_gb), t_bg = event_threshold(c.p_bg);
  const uint64_t t_lg = event_threshold(c.loss_good), t_lb = event_threshold(c.loss_bad);
  const int n = L * P, words = (n + 31) / 32;
  for (int k = lane; k < words; k += kWave) arrived[k] = 0u;
  const int per = (n + kWave - 1) / kWave;
  const int a = lane * per < n ? lane * per : n, b = (a + per) < n ? (a + per) : n;
  // pass 1: this run's end state from either start state
  {
    SlotDraws d;
    uint32_t s0 = 0u, s1 = 1u;
    for (int s = a; s < b; ++s) {
      uint32_t ul, um;
      d.get((uint32_t)s, w, k0, k1, ul, um);
      s0 = s0 ? ((uint64_t)um < t_bg ? 0u : 1u) : ((uint64_t)um < t_gb ? 1u : 0u);
      s1 = s1 ? ((uint64_t)um < t_bg ? 0u : 1u) : ((uint64_t)um < t_gb ? 1u : 0u);
    }
    maps[lane] = s0 | (s1 << 1);
  }
  __syncthreads();
  if (lane == 0) {
    uint32_t out[4];
    philox4x32_10(0xffffffffu, w, kSamplerTag, 0u, k0, k1, out);
    uint32_t st = (uint64_t)out[0] < event_threshold(c.p_start_bad) ? 1u : 0u;
    for (int i = 0; i < kWave; ++i) {
      starts[i] = st;
      st = (maps[i] >> st) & 1u;
    }
  }
  __syncthreads();
  // pass 2: erasures from the true start state
  {
    SlotDraws d;
    uint32_t st = starts[lane];
    for (int s = a; s < b; ++s) {
      uint32_t ul, um;
      d.get((uint32_t)s, w, k0, k1, ul, um);
      bool lost = (uint64_t)ul < (st ? t_lb : t_lg);
      if (c.deadline >= 0 && s >= c.deadline) lost = true;
      if (!lost) atomicOr(&arrived[s >> 5], 1u << (s & 31));
      st = st ? ((uint64_t)um < t_bg ? 0u : 1u) : ((uint64_t)um < t_gb ? 1u : 0u);
    }
  }
  __syncthreads();
  uint8_t *row = codes + (int64_t)w * P;
  for (int p = lane; p < P; p += kWave) {
    int code = 0;
    while (code < L) {
      const int s = code * P + p;
      if (!((arrived[s >> 5] >> (s & 31)) & 1u)) break;
      ++code;
    }
    row[p] = (uint8_t)code;
  }
}

void launch_sample_states(const SamplerChannel *channels, int num_states, int P, int L, uint64_t seed,
                          uint8_t *codes, hipStream_t st) {
  if (num_states <= 0) return;
  const size_t lds = sizeof(uint32_t) * (size_t)ceil_div((int64_t)L * P, 32);
  k_sample_states<<<num_states, kWave, lds, st>>>(channels, P, L, (uint32_t)seed, (uint32_t)(seed >> 32), codes);
}

}  // namespace dgs
