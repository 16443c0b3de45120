// Internal: launch wrapper of the median post-filter kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fgs {

// dst = median of the (2r+1) x (2r+1) window of the binary mask src (nonzero =
// foreground), border pixels replicated; 0 <= r <= kMedRadiusMax.  src and dst are
// device buffers of H rows of W bytes, rows src_stride / dst_stride bytes apart.
constexpr int kMedRadiusMax = 7;
hipError_t post_launch_median(const uint8_t* src, int64_t src_stride, uint8_t* dst, int64_t dst_stride, int H,
                              int W, int radius, hipStream_t s);

}  // namespace fgs
