// Workgroup order across the chip's XCDs.  The dispatcher hands the
// workgroup with linear id w (x fastest, then y, then z) to XCD w mod 8, so
// by default each XCD runs every eighth tile.  xcd_block() renumbers the
// workgroups so that XCD k runs one contiguous range of logical ids, in
// order: neighbouring tiles of an image then share an XCD (and its L2) and
// run at about the same time.  The map is a bijection for any grid size.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace sense {

constexpr uint32_t kXcds = 8;

__host__ __device__ constexpr uint32_t xcd_order(uint32_t w, uint32_t total) {
  const uint32_t q = total / kXcds, r = total % kXcds, k = w % kXcds;
  return k * q + (k < r ? k : r) + w / kXcds;
}

// Compile-time check that xcd_order permutes 0 .. total-1.
constexpr bool xcd_order_permutes(uint32_t total) {
  bool seen[4096] = {};
  if (total > 4096) return false;
  for (uint32_t w = 0; w < total; ++w) {
    const uint32_t l = xcd_order(w, total);
    if (l >= total || seen[l]) return false;
    seen[l] = true;
  }
  return true;
}
static_assert(xcd_order_permutes(1) && xcd_order_permutes(7) && xcd_order_permutes(8) && xcd_order_permutes(13) &&
                  xcd_order_permutes(2560) && xcd_order_permutes(4095),
              "xcd_order must be a bijection");

struct BlockId {
  uint32_t x, y, z;
};

__device__ __forceinline__ BlockId xcd_block() {
  const uint32_t gx = gridDim.x, gy = gridDim.y;
  const uint32_t w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const uint32_t l = xcd_order(w, gx * gy * gridDim.z);
  return {l % gx, (l / gx) % gy, l / (gx * gy)};
}

}  // namespace sense
