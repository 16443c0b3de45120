// Static-object detection on the model's masks (the paper's future work, Sec. 6; read
// here as: a pixel is static once the mask has marked it foreground in each of the last
// M frames).  Per pixel a 16-bit run counter, c = mask ? min(c + 1, 65535) : 0, and the
// static mask 255 where c >= M.  One lane per 4 consecutive pixels: the mask word and the
// static word as 32-bit accesses, the counters as 64-bit ones, where the 4 pixels are
// inside and aligned (the planes are 256-byte aligned, so group g starts at pixel 4g);
// the last group of an image whose size is not a multiple of 4 goes pixel by pixel.
#include "fgs_internal.h"

namespace fgs {

namespace {

__device__ __forceinline__ uint32_t run(uint32_t c, uint32_t fg) { return fg ? (c < 65535u ? c + 1u : 65535u) : 0u; }

__global__ __launch_bounds__(256) void static_update_kernel(const uint8_t* __restrict__ mask,
                                                            uint16_t* __restrict__ count,
                                                            uint8_t* __restrict__ out, int64_t npix, uint32_t M) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t p0 = 4 * g;
    if (p0 >= npix) return;
    if (p0 + 4 <= npix) {
        const uint32_t mw = *reinterpret_cast<const uint32_t*>(mask + p0);
        const uint2 cw = *reinterpret_cast<const uint2*>(count + p0);
        uint32_t c[4] = {cw.x & 0xFFFFu, cw.x >> 16, cw.y & 0xFFFFu, cw.y >> 16};
        uint32_t sw = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c[i] = run(c[i], (mw >> (8 * i)) & 0xFFu);
            sw |= (c[i] >= M ? 0xFFu : 0u) << (8 * i);
        }
        *reinterpret_cast<uint2*>(count + p0) = make_uint2(c[0] | (c[1] << 16), c[2] | (c[3] << 16));
        *reinterpret_cast<uint32_t*>(out + p0) = sw;
        return;
    }
    for (int64_t p = p0; p < npix; ++p) {
        const uint32_t c = run(count[p], mask[p]);
        count[p] = (uint16_t)c;
        out[p] = c >= M ? 255 : 0;
    }
}

__global__ void static_clear_kernel(uint16_t* count, uint8_t* out, int64_t npix) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    count[p] = 0;
    out[p] = 0;
}

}  // namespace

hipError_t static_launch_update(const uint8_t* mask, uint16_t* count, uint8_t* out, int64_t npix, uint32_t M,
                                hipStream_t s) {
    const int64_t groups = (npix + 3) / 4;
    hipLaunchKernelGGL(static_update_kernel, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, mask, count,
                       out, npix, M);
    return hipGetLastError();
}

hipError_t static_launch_clear(uint16_t* count, uint8_t* out, int64_t npix, hipStream_t s) {
    hipLaunchKernelGGL(static_clear_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, count, out, npix);
    return hipGetLastError();
}

}  // namespace fgs
