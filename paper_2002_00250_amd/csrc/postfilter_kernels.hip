// Median post-filter of a binary foreground mask.  The base PBAS method smooths
// its output with a median filter; for a mask whose pixels are background (0) or
// foreground (nonzero) the median of an odd window is foreground exactly when more
// than half of the window is, so the filter is a windowed count and a compare.
#include "postfilter.h"

namespace fgs {

namespace {

constexpr int kMedBlock = 256;
constexpr int kMedTW = 256;                         // tile columns
constexpr int kMedPitch = kMedTW + 2 * kMedRadiusMax + 2;  // LDS row pitch, a multiple of 4

// One workgroup filters a kMedTW x TH tile (1-D grid: tile b at column b mod tiles_x,
// row b / tiles_x).  Window pixels outside the image are read at clamped coordinates,
// which repeats the nearest edge pixel.
//  1. Lane c owns column c of the tile and its R-pixel border (columns kMedTW..kMedTW+2R-1
//     go to lanes 0..2R-1 in a second pass).  It issues all TH + 2R byte loads of the
//     column before using any, and forms the column's sums over 2R+1 rows in registers
//     with a running sum (at most 15, one byte each in LDS).
//  2. Lane t then owns TH consecutive output pixels of one tile row (kMedTW / TH lanes per
//     row): it reads the TH + 2R column sums it needs as LDS words and slides a window
//     of 2R+1 of them.
//  3. One TH-byte store per lane when the row segment lies inside the image and the
//     destination rows are TH-byte aligned, else byte stores.
// All counts are exact integers.
template <int R, int TH>
__global__ __launch_bounds__(kMedBlock) void median_mask_kernel(const uint8_t* __restrict__ src, int64_t ss,
                                                                uint8_t* __restrict__ dst, int64_t ds, int H,
                                                                int W, int tiles_x) {
    static_assert(kMedTW == kMedBlock && (TH == 4 || TH == 8 || TH == 16), "TH output pixels per lane");
    constexpr int kLanesPerRow = kMedTW / TH;
    constexpr int kRows = TH + 2 * R;
    constexpr int kN = (2 * R + 1) * (2 * R + 1);
    __shared__ __align__(16) uint8_t colsum[TH][kMedPitch];
    const int bx = (int)(blockIdx.x % (unsigned)tiles_x), by = (int)(blockIdx.x / (unsigned)tiles_x);
    const int x0 = bx * kMedTW, y0 = by * TH;

#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int c = (int)threadIdx.x + pass * kMedBlock;
        if (pass == 1 && c >= kMedTW + 2 * R) break;
        const int gx = min(max(x0 - R + c, 0), W - 1);
        uint32_t v[kRows];
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int gy = min(max(y0 - R + k, 0), H - 1);
            v[k] = src[(int64_t)gy * ss + gx];
        }
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) s += v[k] != 0;
#pragma unroll
        for (int i = 0; i < TH; ++i) {
            s += v[i + 2 * R] != 0;
            colsum[i][c] = (uint8_t)s;
            s -= v[i] != 0;
        }
    }
    __syncthreads();

    const int row = (int)threadIdx.x / kLanesPerRow, seg = ((int)threadIdx.x % kLanesPerRow) * TH;
    const int y = y0 + row;
    if (y >= H) return;
    constexpr int kWords = (TH + 2 * R + 3) / 4;
    uint32_t cw[kWords];
    const uint32_t* lrow = reinterpret_cast<const uint32_t*>(&colsum[row][seg]);
#pragma unroll
    for (int j = 0; j < kWords; ++j) cw[j] = lrow[j];
    auto cs = [&](int k) -> uint32_t { return (cw[k >> 2] >> (8 * (k & 3))) & 0xffu; };
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) s += cs(k);
    uint32_t outw[TH / 4] = {};
#pragma unroll
    for (int i = 0; i < TH; ++i) {
        s += cs(i + 2 * R);
        outw[i >> 2] |= (2 * s > (uint32_t)kN ? 0xffu : 0u) << (8 * (i & 3));
        s -= cs(i);
    }
    const int x = x0 + seg;
    uint8_t* drow = dst + (int64_t)y * ds + x;
    if (x + TH <= W && ((reinterpret_cast<uintptr_t>(dst) | (uintptr_t)ds) & (TH - 1)) == 0) {
        if constexpr (TH == 16)
            *reinterpret_cast<uint4*>(drow) = make_uint4(outw[0], outw[1], outw[2], outw[3]);
        else if constexpr (TH == 8)
            *reinterpret_cast<uint2*>(drow) = make_uint2(outw[0], outw[1]);
        else
            *reinterpret_cast<uint32_t*>(drow) = outw[0];
    } else {
#pragma unroll
        for (int i = 0; i < TH; ++i)
            if (x + i < W) drow[i] = (uint8_t)(outw[i >> 2] >> (8 * (i & 3)));
    }
}

template <int R>
hipError_t launch_radius(const uint8_t* src, int64_t ss, uint8_t* dst, int64_t ds, int H, int W, hipStream_t s) {
    constexpr int TH = 16;
    const int64_t tiles_x = ((int64_t)W + kMedTW - 1) / kMedTW;
    const int64_t tiles = tiles_x * (((int64_t)H + TH - 1) / TH);
    if (tiles == 0) return hipSuccess;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((median_mask_kernel<R, TH>), dim3((unsigned)tiles), dim3(kMedBlock), 0, s, src, ss, dst,
                       ds, H, W, (int)tiles_x);
    return hipGetLastError();
}

}  // namespace

hipError_t post_launch_median(const uint8_t* src, int64_t src_stride, uint8_t* dst, int64_t dst_stride, int H,
                              int W, int radius, hipStream_t s) {
    static_assert(kMedRadiusMax == 7, "one instantiation per radius");
    switch (radius) {
        case 0: return launch_radius<0>(src, src_stride, dst, dst_stride, H, W, s);
        case 1: return launch_radius<1>(src, src_stride, dst, dst_stride, H, W, s);
        case 2: return launch_radius<2>(src, src_stride, dst, dst_stride, H, W, s);
        case 3: return launch_radius<3>(src, src_stride, dst, dst_stride, H, W, s);
        case 4: return launch_radius<4>(src, src_stride, dst, dst_stride, H, W, s);
        case 5: return launch_radius<5>(src, src_stride, dst, dst_stride, H, W, s);
        case 6: return launch_radius<6>(src, src_stride, dst, dst_stride, H, W, s);
        case 7: return launch_radius<7>(src, src_stride, dst, dst_stride, H, W, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fgs
