// Deterministic block reductions in fp64: a fixed butterfly inside each
// 64-lane wavefront, then wave partials summed in wave order by thread 0.
#pragma once

#include <hip/hip_runtime.h>

namespace sense {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Returns the block total in thread 0 (other threads: unspecified).
// scratch must hold blockDim.x / 64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  static_assert(NT % 64 == 0, "block must be whole wavefronts");
  constexpr int W = NT / 64;
  v = wave_sum(v);
  if constexpr (W == 1) {
    return v;
  } else {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < W; ++i) s += scratch[i];
    }
    return s;
  }
}

// Sum of n partials in a fixed order, the same in every block: in index
// order for n <= 64; above that lane l sums p[l], p[l + 64], ... in index
// order and the 64 lane sums go through the fixed butterfly.  All 64 lanes
// of the calling wavefront must be active.
__device__ __forceinline__ double ordered_sum(const double* __restrict__ p, int n) {
  if (n <= 64) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += p[i];
    return s;
  }
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  // eight loads in flight per lane, added in index order
  for (int i0 = lane; i0 < n; i0 += 64 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = i0 + 64 * u < n ? p[i0 + 64 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  return wave_sum(s);
}

__device__ __forceinline__ bool finite64(double v) { return __builtin_isfinite(v); }

}  // namespace sense
