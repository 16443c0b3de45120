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

__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace

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
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 16) blocks = 256 * 16;  // grid-stride: 16 workgroups per CU
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n);
    return hipGetLastError();
}

}  // namespace fgs
