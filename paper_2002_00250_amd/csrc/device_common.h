// Device helpers shared by the GMM and PBAS kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fgs {

// 8-bit depth code (Sec. 4.1-4.2): 0 = no depth; otherwise the round-half-up
// rescale of millimetres to `full_scale_mm`, clamped to [1, 255].
__device__ __forceinline__ uint32_t depth_code(uint32_t d_mm, uint32_t full_scale_mm) {
    if (d_mm == 0u) return 0u;
    uint32_t q = (__umul24(255u, d_mm) + (full_scale_mm >> 1)) / full_scale_mm;  // d_mm < 2^16
    q = q < 1u ? 1u : q;
    return q > 255u ? 255u : q;
}

// Depth (mm) seen by RGB pixel (x, y).  The depth map is either W x H, or dw x dh
// and brought to the RGB grid by nearest-neighbour upscaling on pixel centres
// (Sec. 4.3: depth is upscaled to the RGB resolution when the two differ):
// xd = floor((x + 1/2) dw / W), yd = floor((y + 1/2) dh / H).
__device__ __forceinline__ uint32_t load_depth(const uint8_t* depth, int64_t stride, int x, int y,
                                               int W, int H, int dw, int dh) {
    int xd = x, yd = y;
    if (dw > 0) {
        xd = (int)(((int64_t)(2 * x + 1) * dw) / (2 * (int64_t)W));
        yd = (int)(((int64_t)(2 * y + 1) * dh) / (2 * (int64_t)H));
    }
    return *reinterpret_cast<const uint16_t*>(depth + (int64_t)yd * stride + 2 * xd);
}

struct U32x4 {
    uint32_t v[4];
};

// a ^ b ^ k in one instruction (the three-input bitwise operation, truth table 0x96); k is
// wave-uniform (the generator's key words)
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "s"(k));
    return d;
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the keyed bijection on a
// 128-bit counter.  Each round forms the two 64-bit products of counter words
// 0 and 2 with the round multipliers and permutes their halves with words 1
// and 3 and the key; the key advances by the Weyl increments between rounds.
__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // (round 0's words 1 and 3 are the caller's, often constants: left to the compiler)
        const uint32_t n0 = r == 0 ? (uint32_t)(p1 >> 32) ^ c1 ^ k0 : xor3_key((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = r == 0 ? (uint32_t)(p0 >> 32) ^ c3 ^ k1 : xor3_key((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    U32x4 r;
    r.v[0] = c0;
    r.v[1] = c1;
    r.v[2] = c2;
    r.v[3] = c3;
    return r;
}

}  // namespace fgs
