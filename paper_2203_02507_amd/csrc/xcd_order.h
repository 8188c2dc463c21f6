// XCD-aware order of a launch's items (HIP device code only).
//
// The GPU hands workgroup b of a launch to XCD b mod kXcds, so a launch whose
// items are grouped by tile deals them out in kXcds contiguous blocks, one
// per XCD: the LED-group members of a tile then run on one XCD and read the
// tile's pupil from that XCD's L2.  The grid is xcd_grid(count) workgroups;
// xcd_item returns -1 for the few workgroups past the last item.
#pragma once

#include <hip/hip_runtime.h>

namespace fpm {

constexpr int kXcds = 8;

__host__ __device__ constexpr int xcd_grid(int count) {
  return (count + kXcds - 1) / kXcds * kXcds;
}

__device__ __forceinline__ int xcd_item(int b, int count) {
  const int per = (count + kXcds - 1) / kXcds;
  const int ii = (b % kXcds) * per + b / kXcds;
  return ii < count ? ii : -1;
}

}  // namespace fpm
