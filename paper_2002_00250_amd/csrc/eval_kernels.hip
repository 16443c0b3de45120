// Evaluation counters (Sec. 5): the confusion counts of a mask against a
// ground-truth mask, accumulated on the device so that a sequence can be scored
// without a host round trip per frame.
#include "fgs_internal.h"

namespace fgs {

namespace {

constexpr int kEvalBlock = 256;
constexpr int kEvalGroup = 4;  // consecutive pixels of one row per lane and step

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Counters are spread over kEvalSlots slots each (workgroup b adds to slot
// b mod kEvalSlots) so that concurrent atomics rarely meet on one address; the
// reader sums the slots.
// acc[c * kEvalSlots + slot], c = TP, TN, FP, FN, of mask (H x W, rows W bytes
// apart) against gt (rows gt_stride bytes apart); nonzero = foreground.  Grid-
// stride over groups of 4 pixels of a row; a wavefront then a workgroup reduction,
// and one 64-bit atomic add per counter and workgroup.
__global__ __launch_bounds__(kEvalBlock) void eval_count_kernel(const uint8_t* __restrict__ mask,
                                                                const uint8_t* __restrict__ gt,
                                                                int64_t gt_stride, int H, int W,
                                                                unsigned long long* __restrict__ acc) {
    __shared__ uint32_t part[kEvalBlock / 64][4];
    const int gpr = (W + kEvalGroup - 1) / kEvalGroup;  // groups per row
    const int64_t total = (int64_t)gpr * H;
    uint32_t tp = 0, fp = 0, fn = 0, n = 0;
    for (int64_t g = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kEvalBlock) {
        const int y = (int)(g / gpr);
        const int x0 = (int)(g - (int64_t)y * gpr) * kEvalGroup;
        const uint8_t* mr = mask + (int64_t)y * W;
        const uint8_t* gr = gt + (int64_t)y * gt_stride;
#pragma unroll
        for (int i = 0; i < kEvalGroup; ++i) {
            const int x = x0 + i;
            if (x < W) {
                const uint32_t m = mr[x] != 0, t = gr[x] != 0;
                tp += m & t;
                fp += m & (t ^ 1u);
                fn += (m ^ 1u) & t;
                n += 1;
            }
        }
    }
    tp = wave_sum(tp);
    fp = wave_sum(fp);
    fn = wave_sum(fn);
    n = wave_sum(n);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[wave][0] = tp;
        part[wave][1] = n - tp - fp - fn;
        part[wave][2] = fp;
        part[wave][3] = fn;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        unsigned long long v = 0;
#pragma unroll
        for (int w = 0; w < kEvalBlock / 64; ++w) v += part[w][threadIdx.x];
        if (v != 0) atomicAdd(acc + threadIdx.x * kEvalSlots + (blockIdx.x % kEvalSlots), v);
    }
}

// Clears the accumulator (a kernel rather than a memset, so the call may sit in a
// captured graph).
__global__ void eval_zero_kernel(unsigned long long* acc) {
    acc[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t eval_launch_count(const uint8_t* mask, const uint8_t* gt, int64_t gt_stride, int H, int W,
                             unsigned long long* acc, hipStream_t s) {
    const int64_t groups = (int64_t)((W + kEvalGroup - 1) / kEvalGroup) * H;
    int64_t blocks = (groups + kEvalBlock - 1) / kEvalBlock;
    if (blocks > 512) blocks = 512;  // 2 per CU; lanes then loop
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(eval_count_kernel, dim3((unsigned)blocks), dim3(kEvalBlock), 0, s, mask, gt, gt_stride,
                       H, W, acc);
    return hipGetLastError();
}

hipError_t eval_launch_zero(unsigned long long* acc, hipStream_t s) {
    hipLaunchKernelGGL(eval_zero_kernel, dim3(1), dim3(4 * kEvalSlots), 0, s, acc);
    return hipGetLastError();
}

}  // namespace fgs
