// Workgroup-level building blocks shared by the split, build and probe
// kernels.
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

// 16-bit half i of a packed array (half i & 1 of word i >> 1).
__device__ __forceinline__ uint32_t get_half(const uint32_t* a, uint32_t i) {
  return (a[i >> 1] >> ((i & 1u) << 4)) & 0xFFFFu;
}

}  // namespace hg
