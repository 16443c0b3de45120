// Diagnostic kernels: the Philox4x32-10 generator PBAS draws from, exposed on
// its own so it can be checked word for word, and a plain streaming copy that
// calibrates the HBM bandwidth a simple kernel reaches on this device.
#include "device_common.h"
#include "fgs_internal.h"

namespace fgs {

namespace {

__global__ void philox_kernel(uint32_t k0, uint32_t k1, const uint4* __restrict__ ctr,
                              uint4* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = ctr[i];
    const U32x4 r = philox4x32_10(c.x, c.y, c.z, c.w, k0, k1);
    out[i] = make_uint4(r.v[0], r.v[1], r.v[2], r.v[3]);
}

// One 16-byte element per lane, non-temporal: the fastest plain copy shape measured on
// this device (6.6 TB/s; two or four elements per lane 6.2-6.4, eight 4.2).
__global__ __launch_bounds__(256) void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   int64_t n) {
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        __builtin_nontemporal_store(__builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src) + i),
                                    reinterpret_cast<u32x4*>(dst) + i);
}

// Read/write mixes of the step kernels' shape: one lane per pixel reads RP float4
// planes and writes the first WP of them back in place, non-temporal like the step
// kernels' state traffic (the value written depends on every value read).
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int RP, int WP>
__global__ __launch_bounds__(256) void mix_kernel(f32x4* __restrict__ planes, int64_t npix) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    f32x4 v[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) v[i] = __builtin_nontemporal_load(planes + (int64_t)i * npix + p);
    f32x4 acc = v[0];
#pragma unroll
    for (int i = 1; i < RP; ++i) acc += v[i];
#pragma unroll
    for (int i = 0; i < WP; ++i) {
        f32x4 o = v[i];
        o.x = acc.x * 0.5f + 1.0f;
        __builtin_nontemporal_store(o, planes + (int64_t)i * npix + p);
    }
    if (WP == 0 && acc.x == -1.0f) planes[p] = acc;  // (keeps the reads of a read-only mix)
}

template <int WP>
__global__ __launch_bounds__(256) void write_only_kernel(f32x4* __restrict__ planes, int64_t npix) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const f32x4 o = {(float)p, 1.0f, 2.0f, 3.0f};
#pragma unroll
    for (int i = 0; i < WP; ++i) __builtin_nontemporal_store(o, planes + (int64_t)i * npix + p);
}

}  // namespace

hipError_t diag_launch_mix(void* planes, int64_t npix, int mode, hipStream_t s) {
    if (npix <= 0) return hipSuccess;
    const dim3 grid((unsigned)((npix + 255) / 256)), block(256);
    f32x4* pl = reinterpret_cast<f32x4*>(planes);
    switch (mode) {
        case 0: hipLaunchKernelGGL((mix_kernel<10, 10>), grid, block, 0, s, pl, npix); break;
        case 1: hipLaunchKernelGGL((mix_kernel<10, 5>), grid, block, 0, s, pl, npix); break;
        case 2: hipLaunchKernelGGL((mix_kernel<10, 0>), grid, block, 0, s, pl, npix); break;
        case 3: hipLaunchKernelGGL((write_only_kernel<10>), grid, block, 0, s, pl, npix); break;
        case 4: hipLaunchKernelGGL((mix_kernel<9, 9>), grid, block, 0, s, pl, npix); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t diag_launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32),
                       reinterpret_cast<const uint4*>(ctr), reinterpret_cast<uint4*>(out), n);
    return hipGetLastError();
}

hipError_t diag_launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n);
    return hipGetLastError();
}

}  // namespace fgs
