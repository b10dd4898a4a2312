// Workgroup- and wave-level building blocks shared by the split, build and
// probe kernels.
#pragma once

#include "hg_device.h"

namespace hg {

// Exclusive sum over a workgroup of THREADS threads; `total` receives the sum
// of all values.  wtot holds THREADS / 64 words of LDS.  Every thread of the
// workgroup must call it (it contains barriers).
template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t* wtot, uint32_t& total) {
  constexpr int kW = THREADS / kWave;
  const uint32_t inc = wave_inclusive_sum(v);
  const uint32_t w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) wtot[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int x = 0; x < kW; ++x) {
    const uint32_t c = wtot[x];
    base += (x < static_cast<int>(w)) ? c : 0u;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return base + inc - v;
}

// Wave-level multisplit (a ballot per digit bit, as in Ashkiani et al.,
// "GPU Multisplit", PPoPP 2016).  For item i of every lane the lanes holding
// the same digit form `match`; the lowest of them adds the group size to the
// wave's private counter of that digit with one LDS atomic and hands the old
// value to the group.  LDS executes a wave's operations in issue order, so
// the atomics of consecutive items need not wait for each other, and the
// resulting order, (item, lane), is deterministic: an inverse pass recomputes
// it exactly.  wcnt packs two 16-bit counters per word (digit d in half d & 1
// of word d >> 1; a wave never counts more than 64 * ITEMS < 2^16 keys).
template <int ITEMS>
__device__ __forceinline__ void wave_multisplit(const uint32_t (&d)[ITEMS], uint32_t mask, uint32_t nbits,
                                                uint32_t* wcnt, uint32_t (&rank)[ITEMS]) {
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const bool valid = (mask >> i) & 1u;
    uint64_t match = ballot(valid);
    for (uint32_t b = 0; b < nbits; ++b) {
      const bool bit = (d[i] >> b) & 1u;
      const uint64_t bb = ballot(bit);
      match &= bit ? bb : ~bb;
    }
    const uint32_t below = popc64(match & lt);
    const uint32_t sh = (d[i] & 1u) << 4;
    uint32_t prior = 0;
    if (valid && below == 0) prior = (atomicAdd(&wcnt[d[i] >> 1], popc64(match) << sh) >> sh) & 0xFFFFu;
    const uint32_t leader = valid ? static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(match)) - 1)
                                  : lane_id();
    prior = __shfl(prior, static_cast<int>(leader), kWave);
    rank[i] = prior + below;
  }
}

__device__ __forceinline__ uint32_t get_half(const uint32_t* a, uint32_t i) {
  return (a[i >> 1] >> ((i & 1u) << 4)) & 0xFFFFu;
}

__device__ __forceinline__ void set_half(uint32_t* a, uint32_t i, uint32_t v) {
  const uint32_t sh = (i & 1u) << 4;
  a[i >> 1] = (a[i >> 1] & ~(0xFFFFu << sh)) | (v << sh);
}

// Number of bits needed for digits 0 .. D-1.
__device__ __forceinline__ uint32_t digit_bits(uint32_t D) { return D <= 1 ? 0u : 32u - __clz(D - 1); }

}  // namespace hg
