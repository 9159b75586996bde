// Device helpers shared by the kernel sources (wave size, wave reductions)
// and the grid-size helper of their launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WAVE));
  return v;
}

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace hm
