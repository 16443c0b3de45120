// RGB-D Pixel-Based Adaptive Segmenter kernels (Sec. 3.2): one launch per frame
// (fill for the first N frames, then the tile update of pbas_device.h), the
// flush of pending neighbour writes before a state read-out, and the state
// import/export.
#include <cstring>

#include "device_common.h"
#include "fgs_internal.h"
#include "pbas_device.h"

namespace fgs {

using namespace pbas;

namespace {

// Frames 0..N-1: sample slot t takes the frame; the mask is empty.
__global__ __launch_bounds__(256) void pbas_fill_kernel(PbasStepArgs a) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < a.npix) fill_pixel(a, p);
}

// Register capacity class NMAX serves N in [class_min(NMAX), NMAX].
constexpr int class_min(int nmax) { return nmax <= 8 ? 2 : (nmax <= 40 ? nmax - 3 : nmax - 7); }

// One block per 64x4 tile on a one-dimensional grid (row-major tile order within a
// model): the grid's y extent is too small for the tile rows of a tall image.  One
// launch steps b.n models (one for a single push): workgroup w takes tile
// w - first[i] of model i, first[i] <= w < first[i + 1].
template <int NB, int NMAX, bool NT>
__global__ __launch_bounds__(kBlock) void pbas_step_kernel(PbasBatch<NB> b) {
    __shared__ PbasLds<NMAX> sh;
    const int w = (int)blockIdx.x;
    int i = 0;
#pragma unroll
    for (int j = 1; j < NB; ++j) i += (j < b.n && w >= b.first[j]) ? 1 : 0;
    const int local = w - b.first[i], tiles_x = b.tiles_x[i];
    pbas_tile<NMAX, class_min(NMAX), NT>(b.a[i], local % tiles_x, local / tiles_x, sh);
}

// Apply the neighbour writes of the last processed frame (read-out of the logical
// state): each pixel looks at its 8 neighbours; a neighbour q in direction d that
// fired recomputes its draws and counts if it aimed the opposite way, 7 - d (the
// direction table is point symmetric).  Writes carry the pixel's own value of that
// frame; the depth channel only where the pixel had depth.
__global__ __launch_bounds__(256) void pbas_flush_kernel(PbasPlanes m, int H, int W, uint32_t t_prev,
                                                         int N, uint32_t k0, uint32_t k1) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= H * W) return;
    const int y = p / W, x = p - y * W;
    const int64_t npix = (int64_t)H * W;
    const uint32_t lastw = m.last_in_pad ? *reinterpret_cast<const uint32_t*>(sample_byte(m.samples, npix, N, p, 0))
                                         : m.last[p];
    const uint8_t* fire = m.fire[t_prev & 1u];
    for (int d = 0; d < 8; ++d) {
        const int qx = x + nb_dx(d), qy = y + nb_dy(d);
        if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
        const int q = qy * W + qx;
        const uint32_t fb = fire[q] & 0xFu;  // channels that fired (the high nibble: R flags)
        if (fb == 0u) continue;
        const U32x4 w1 = philox4x32_10((uint32_t)q, t_prev, 1u, 0u, k0, k1);
        for (int j = 0; j < 4; ++j) {
            if (!((fb >> j) & 1u)) continue;
            int dq, slot;
            intent_of(w1.v[j], N, dq, slot);
            const uint32_t val = (lastw >> (8 * j)) & 0xFFu;
            if (dq != 7 - d || (j == 3 && val == 0u)) continue;
            *sample_byte(m.samples, npix, slot, p, j) = (uint8_t)val;
        }
    }
}

__global__ void pbas_init_state_kernel(PbasPlanes m, int npix, float4 Rl, float Tl) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    m.R[p] = Rl;
    m.T[p] = make_float4(Tl, Tl, Tl, Tl);
}

// Canonical R[4], T[4] float32 planes and S[4] uint16 planes <-> per-pixel vectors.
__global__ void pbas_export_rts_kernel(PbasPlanes m, int npix, float* rt, uint16_t* s) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    const float4 r = m.R[p], t = m.T[p];
    const uint2 sv = m.S[p];
    rt[0 * n + p] = r.x; rt[1 * n + p] = r.y; rt[2 * n + p] = r.z; rt[3 * n + p] = r.w;
    rt[4 * n + p] = t.x; rt[5 * n + p] = t.y; rt[6 * n + p] = t.z; rt[7 * n + p] = t.w;
    s[0 * n + p] = (uint16_t)(sv.x & 0xFFFFu);
    s[1 * n + p] = (uint16_t)(sv.x >> 16);
    s[2 * n + p] = (uint16_t)(sv.y & 0xFFFFu);
    s[3 * n + p] = (uint16_t)(sv.y >> 16);
}

__global__ void pbas_import_rts_kernel(PbasPlanes m, int npix, const float* rt, const uint16_t* s) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    m.R[p] = make_float4(rt[0 * n + p], rt[1 * n + p], rt[2 * n + p], rt[3 * n + p]);
    m.T[p] = make_float4(rt[4 * n + p], rt[5 * n + p], rt[6 * n + p], rt[7 * n + p]);
    m.S[p] = make_uint2((uint32_t)s[0 * n + p] | ((uint32_t)s[1 * n + p] << 16),
                        (uint32_t)s[2 * n + p] | ((uint32_t)s[3 * n + p] << 16));
}

// Canonical slot-major sample planes (plane k = slot k of every pixel) <-> the
// device's quad planes.  Import writes the padding slots as zero.
__global__ void pbas_export_samples_kernel(const uint4* quads, uint32_t* out, int npix, int N) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    for (int q = 0; 4 * q < N; ++q) {
        const uint4 v = quads[q * n + p];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        for (int i = 0; i < 4 && 4 * q + i < N; ++i) out[(4 * q + i) * n + p] = w[i];
    }
}

__global__ void pbas_import_samples_kernel(uint4* quads, const uint32_t* in, int npix, int N) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    for (int q = 0; 4 * q < N; ++q) {
        uint32_t w[4];
        for (int i = 0; i < 4; ++i) w[i] = 4 * q + i < N ? in[(4 * q + i) * n + p] : 0u;
        quads[q * n + p] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

inline unsigned blocks1d(int n) { return (unsigned)((n + 255) / 256); }

template <int NB, int NMAX>
void launch_step_nt(const PbasBatch<NB>& b, dim3 grid, hipStream_t s) {
    if (b.a[0].streaming) hipLaunchKernelGGL((pbas_step_kernel<NB, NMAX, true>), grid, dim3(kBlock), 0, s, b);
    else hipLaunchKernelGGL((pbas_step_kernel<NB, NMAX, false>), grid, dim3(kBlock), 0, s, b);
}

// Register capacity for the N sample words: the smallest instantiated NMAX >= N
// (multiples of 4 up to 40, then 48, 56, 64), so that N >= class_min(NMAX).
int nmax_class(int N) {
    switch ((N + 3) / 4) {
        case 0: case 1: case 2: return 8;
        case 11: case 12: return 48;
        case 13: case 14: return 56;
        default: return (N + 3) / 4 <= 10 ? 4 * ((N + 3) / 4) : 64;
    }
}

template <int NB>
void launch_step_n(const PbasBatch<NB>& b, dim3 grid, hipStream_t s) {
    switch (nmax_class(b.a[0].c.N)) {
        case 8: launch_step_nt<NB, 8>(b, grid, s); break;
        case 12: launch_step_nt<NB, 12>(b, grid, s); break;
        case 16: launch_step_nt<NB, 16>(b, grid, s); break;
        case 20: launch_step_nt<NB, 20>(b, grid, s); break;
        case 24: launch_step_nt<NB, 24>(b, grid, s); break;
        case 28: launch_step_nt<NB, 28>(b, grid, s); break;
        case 32: launch_step_nt<NB, 32>(b, grid, s); break;
        case 36: launch_step_nt<NB, 36>(b, grid, s); break;
        case 40: launch_step_nt<NB, 40>(b, grid, s); break;
        case 48: launch_step_nt<NB, 48>(b, grid, s); break;
        case 56: launch_step_nt<NB, 56>(b, grid, s); break;
        default: launch_step_nt<NB, 64>(b, grid, s); break;
    }
}

template <int NB>
hipError_t launch_batch(const PbasStepArgs* a, int n, hipStream_t s) {
    PbasBatch<NB> b;
    std::memset(&b, 0, sizeof b);
    b.n = n;
    int64_t grid = 0;
    for (int i = 0; i < n; ++i) {
        b.a[i] = a[i];
        b.tiles_x[i] = (a[i].W + kTileW - 1) / kTileW;
        b.first[i] = (int32_t)grid;
        // ceil(W/64) * ceil(H/4) <= H*W/256 + W/64 + H/4 + 1 < 2^27 tiles for H*W <= 2^28
        grid += (int64_t)b.tiles_x[i] * ((a[i].H + kTileH - 1) / kTileH);
    }
    for (int i = n; i <= NB; ++i) b.first[i] = (int32_t)grid;
    for (int i = n; i < NB; ++i) b.tiles_x[i] = 1;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    launch_step_n(b, dim3((unsigned)grid), s);
    return hipGetLastError();
}

}  // namespace

hipError_t pbas_launch_init_state(const PbasPlanes& m, int npix, const PbasConsts& c,
                                  hipStream_t s) {
    hipLaunchKernelGGL(pbas_init_state_kernel, dim3(blocks1d(npix)), dim3(256), 0, s, m, npix,
                       make_float4(c.R_lower[0], c.R_lower[1], c.R_lower[2], c.R_lower[3]),
                       c.T_lower);
    return hipGetLastError();
}

int pbas_batch_key(const PbasStepArgs& a) {
    if ((int)a.t < a.c.N) return -1;
    return nmax_class(a.c.N) * 2 + (a.streaming ? 1 : 0);
}

hipError_t pbas_launch_step_batch(const PbasStepArgs* a, int n, hipStream_t s) {
    if (n < 1 || n > kBatchMax) return hipErrorInvalidValue;
    for (int i = 0; i < n; ++i) {
        const int key = pbas_batch_key(a[i]);
        if (key < 0 || key != pbas_batch_key(a[0])) return hipErrorInvalidValue;
    }
    return n == 1 ? launch_batch<1>(a, n, s) : launch_batch<kBatchMax>(a, n, s);
}

hipError_t pbas_launch_step(const PbasStepArgs& a, hipStream_t s) {
    if (pbas_batch_key(a) < 0) {
        hipLaunchKernelGGL(pbas_fill_kernel, dim3(blocks1d(a.npix)), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    return pbas_launch_step_batch(&a, 1, s);
}

hipError_t pbas_launch_flush(const PbasPlanes& m, int H, int W, uint32_t t_prev, const PbasConsts& c,
                             hipStream_t s) {
    hipLaunchKernelGGL(pbas_flush_kernel, dim3(blocks1d(H * W)), dim3(256), 0, s, m, H, W, t_prev, c.N,
                       c.key0, c.key1);
    return hipGetLastError();
}

// Canonical payload: samples[N] u32, dhist[N] u32, R[4] f32, T[4] f32, S[4] u16
// (out and in are 4-byte aligned device buffers).
hipError_t pbas_launch_export(const PbasPlanes& m, int npix, int N, uint8_t* out, hipStream_t s) {
    const size_t plane = (size_t)npix * 4;
    hipLaunchKernelGGL(pbas_export_samples_kernel, dim3(blocks1d(npix)), dim3(256), 0, s,
                       reinterpret_cast<const uint4*>(m.samples), reinterpret_cast<uint32_t*>(out), npix, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(out + plane * N, m.dhist, plane * N, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    float* rt = reinterpret_cast<float*>(out + 2 * plane * N);
    uint16_t* sv = reinterpret_cast<uint16_t*>(out + 2 * plane * N + 8 * plane);
    hipLaunchKernelGGL(pbas_export_rts_kernel, dim3(blocks1d(npix)), dim3(256), 0, s, m, npix, rt, sv);
    return hipGetLastError();
}

hipError_t pbas_launch_import(const PbasPlanes& m, int npix, int N, const uint8_t* in,
                              hipStream_t s) {
    const size_t plane = (size_t)npix * 4;
    hipLaunchKernelGGL(pbas_import_samples_kernel, dim3(blocks1d(npix)), dim3(256), 0, s,
                       reinterpret_cast<uint4*>(m.samples), reinterpret_cast<const uint32_t*>(in), npix, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(m.dhist, in + plane * N, plane * N, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    const float* rt = reinterpret_cast<const float*>(in + 2 * plane * N);
    const uint16_t* sv = reinterpret_cast<const uint16_t*>(in + 2 * plane * N + 8 * plane);
    hipLaunchKernelGGL(pbas_import_rts_kernel, dim3(blocks1d(npix)), dim3(256), 0, s, m, npix, rt, sv);
    return hipGetLastError();
}

}  // namespace fgs
