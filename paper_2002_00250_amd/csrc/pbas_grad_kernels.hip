// RGB-D PBAS with the base method's gradient-magnitude feature on the colour channels
// (opt-in; Sec. 3.2's RGB-D variant leaves it out).  Per colour channel j a sample slot
// holds the value v and the gradient magnitude m = (|gx| + |gy|) >> 3 of that channel's
// plane (3x3 Sobel, border replicated), and
//   dist = w_j * |m - B^m| + |v - B^v|   (float32, in that order, no contraction)
//   w_j  = alpha / max(mean of m_j over the previous frame, 1)
// with d_min, D and S in float32; the depth channel keeps the integer value distance.
// Everything else (fill frames, classification by match count, self-update, deferred
// neighbour update through fire bytes and the LDS scatter of pbas_device.h, R and T) is
// the plain variant's, so the random draws and decisions follow the same rules.
//
// Layout (fgs_internal.h, PbasGradPlanes): plain slot planes rather than the plain
// variant's quad planes.  This variant trades speed for the second feature: every
// slot's two words are read per frame and a changed slot is written back by word.
#include <cstring>

#include "device_common.h"
#include "fgs_internal.h"
#include "pbas_device.h"

namespace fgs {

using namespace pbas;

namespace {

constexpr int kGradNmax = 64;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// The three colour magnitudes of pixel (x, y) as bytes m_R | m_G << 8 | m_B << 16.
__device__ __forceinline__ uint32_t colour_magnitudes(const uint8_t* rgb, int64_t stride, int x, int y, int W,
                                                      int H) {
    int v[3][3][3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        const uint8_t* row = rgb + (int64_t)clampi(y + dy - 1, 0, H - 1) * stride;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const uint8_t* px = row + 3 * clampi(x + dx - 1, 0, W - 1);
#pragma unroll
            for (int j = 0; j < 3; ++j) v[dy][dx][j] = px[j];
        }
    }
    uint32_t out = 0u;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int gx = (v[0][2][j] + 2 * v[1][2][j] + v[2][2][j]) - (v[0][0][j] + 2 * v[1][0][j] + v[2][0][j]);
        const int gy = (v[2][0][j] + 2 * v[2][1][j] + v[2][2][j]) - (v[0][0][j] + 2 * v[0][1][j] + v[0][2][j]);
        out |= (uint32_t)((abs(gx) + abs(gy)) >> 3) << (8 * j);
    }
    return out;
}

// Adds the block's colour magnitudes to frame t's sums (one 64-bit atomic per channel
// and block; integer sums, so the order does not matter), and block 0 clears frame
// t+1's slot, which nothing reads or writes during frame t.
__device__ __forceinline__ void add_magnitudes(unsigned long long* gsum, uint32_t t, uint32_t mw, bool inside) {
    __shared__ uint32_t part[kBlock / 64][3];
    uint32_t c[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        uint32_t v = inside ? (mw >> (8 * j)) & 0xFFu : 0u;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        c[j] = v;
    }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < 3; ++j) part[threadIdx.x >> 6][j] = c[j];
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) v += part[w][threadIdx.x];
        if (v) atomicAdd(gsum + 4 * (t % 3u) + threadIdx.x, v);
        if (blockIdx.x == 0) gsum[4 * (((uint64_t)t + 1u) % 3u) + threadIdx.x] = 0ull;
    }
}

__device__ __forceinline__ uint32_t frame_word(const PbasGradArgs& a, int x, int y, bool& valid) {
    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = load_depth(a.depth, a.depth_stride, x, y, a.W, a.H, a.depth_w, a.depth_h);
    valid = dmm > 0u;
    return (uint32_t)px[0] | ((uint32_t)px[1] << 8) | ((uint32_t)px[2] << 16) |
           (depth_code(dmm, a.c.depth_max_mm) << 24);
}

// Frames 0..N-1: slot t takes the frame's value and magnitudes; the mask is empty.
__global__ __launch_bounds__(kBlock) void pbas_grad_fill_kernel(PbasGradArgs a) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    const bool inside = p < a.npix;
    const int q = inside ? p : 0;
    const int y = q / a.W, x = q - y * a.W;
    bool valid;
    const uint32_t v = frame_word(a, x, y, valid);
    const uint32_t mw = colour_magnitudes(a.rgb, a.rgb_stride, x, y, a.W, a.H);
    add_magnitudes(a.m.gsum, a.t, mw, inside);
    if (!inside) return;
    const int64_t o = (int64_t)a.t * a.npix + p;
    a.m.samples[o] = v;
    a.m.gsamples[o] = mw;
    a.m.last[p] = v;
    a.m.last_g[p] = mw;
    a.m.mask[p] = 0;
}

// One updating frame on a 64x4 tile (the plain variant's tiling, so the fire-byte
// halo and the LDS scatter of pending neighbour writes are shared).
__global__ __launch_bounds__(kBlock) void pbas_grad_step_kernel(PbasGradArgs a) {
    __shared__ PbasLds<kGradNmax> sh;
    constexpr int NW = PbasLds<kGradNmax>::NW;
    const int tid = threadIdx.x;
    const int tiles_x = (a.W + kTileW - 1) / kTileW;
    const int bx = (int)blockIdx.x % tiles_x, by = (int)blockIdx.x / tiles_x;
    const int x0 = bx * kTileW, y0 = by * kTileH;
    const int lx = tid % kTileW, ly = tid / kTileW;
    const bool inside = x0 + lx < a.W && y0 + ly < a.H;
    const int x = inside ? x0 + lx : x0, y = inside ? y0 + ly : y0;
    const int p = y * a.W + x;
    const int64_t npix = a.npix;
    const int N = a.c.N;

    FireIn fin = {{0u, 0u}, {0, 0}};
    if (a.apply_pending) {
#pragma unroll
        for (int w = 0; w < NW; ++w) sh.pend[w * kBlock + tid] = 0u;
        fin = load_fire(a.m.fire[(a.t - 1u) & 1u], x0, y0, a.H, a.W);
    }
    bool valid;
    const uint32_t Iw = frame_word(a, x, y, valid);
    const uint32_t Mw = colour_magnitudes(a.rgb, a.rgb_stride, x, y, a.W, a.H);
    // weights from the previous frame's magnitude sums
    float wgt[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const unsigned long long sum = a.m.gsum[4 * (((uint64_t)a.t + 2u) % 3u) + j];  // frame t-1's slot
        const float mean = (float)(double)sum / (float)a.npix;
        wgt[j] = a.c.grad_alpha / fmaxf(mean, 1.0f);
    }
    if (a.apply_pending) {
        __syncthreads();  // bit-words cleared
        scatter_fired<kGradNmax>(sh, fin, N, a.t - 1u, a.c.key0, a.c.key1);
        __syncthreads();  // every write aimed at the tile recorded
    }
    add_magnitudes(a.m.gsum, a.t, Mw, inside);  // frame t's sums (after the reads of t-1's slot)
    if (!inside) return;

    const float4 Tv = a.m.T[p], Rv = a.m.R[p], Sv = a.m.S[p];
    float R[4] = {Rv.x, Rv.y, Rv.z, Rv.w};
    float T[4] = {Tv.x, Tv.y, Tv.z, Tv.w};
    float S[4] = {Sv.x, Sv.y, Sv.z, Sv.w};
    const uint32_t lastw = a.m.last[p], lastg = a.m.last_g[p];
    const bool active[4] = {true, true, true, valid};

    // Frame t-1's neighbour writes into this pixel (its previous value and magnitudes)
    // are merged slot by slot, then each slot is classified.
    // (bit-word k >> 3 read from LDS when its first slot comes: a register array
    // indexed by a run-time slot would go to scratch memory)
    const uint32_t keep = (lastw >> 24) != 0u ? 0xFFFFFFFFu : 0x00FFFFFFu;  // depth at t-1?
    int cnt[4] = {0, 0, 0, 0};
    float dmin[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
    uint32_t pw = 0u;
    for (int k = 0; k < N; ++k) {
        const int64_t o = (int64_t)k * npix + p;
        uint32_t s = a.m.samples[o], g = a.m.gsamples[o];
        if ((k & 7) == 0) pw = a.apply_pending ? sh.pend[(k >> 3) * kBlock + tid] & keep : 0u;
        const uint32_t bm = slot_byte_mask(pw, k);
        if (bm) {
            s = (s & ~bm) | (lastw & bm);
            g = (g & ~(bm & 0x00FFFFFFu)) | (lastg & bm & 0x00FFFFFFu);
            a.m.samples[o] = s;
            a.m.gsamples[o] = g;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int dv = abs((int)((s >> (8 * j)) & 0xFFu) - (int)((Iw >> (8 * j)) & 0xFFu));
            const int dm = abs((int)((g >> (8 * j)) & 0xFFu) - (int)((Mw >> (8 * j)) & 0xFFu));
            const float d = wgt[j] * (float)dm + (float)dv;
            cnt[j] += d < R[j] ? 1 : 0;
            dmin[j] = fminf(dmin[j], d);
        }
        const uint32_t sd = s >> 24;
        if (sd != 0u) {  // a depth byte 0 in a sample: nothing recorded
            const float d = (float)abs((int)sd - (int)(Iw >> 24));
            cnt[3] += d < R[3] ? 1 : 0;
            dmin[3] = fminf(dmin[3], d);
        }
    }
    if (dmin[3] == INFINITY) dmin[3] = 255.0f;

    bool F[4];
    bool fg = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        F[j] = active[j] && cnt[j] < a.c.min_matches;
        fg = fg || F[j];
    }
    a.m.mask[p] = fg ? (uint8_t)255 : (uint8_t)0;

    // Self-update with probability 1/T (T from before this frame): slot k of channel j
    // takes the value (and magnitude), its D slot d_min, S = (S - D_k) + d_min.
    const float inv16 = 1.0f / 65536.0f;
    const U32x4 w0 = philox4x32_10((uint32_t)p, a.t, 0u, 0u, a.c.key0, a.c.key1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t a0 = w0.v[j];
        if (!active[j] || F[j] || !((float)(a0 >> 16) * inv16 * T[j] < 1.0f)) continue;
        const int k = (int)(__umul24(a0 & 0xFFFFu, (uint32_t)N) >> 16);
        const int64_t o = (int64_t)k * npix + p;
        reinterpret_cast<uint8_t*>(a.m.samples + o)[j] = (uint8_t)(Iw >> (8 * j));
        if (j < 3) reinterpret_cast<uint8_t*>(a.m.gsamples + o)[j] = (uint8_t)(Mw >> (8 * j));
        float* dk = reinterpret_cast<float*>(a.m.D + o) + j;
        S[j] = (S[j] - *dk) + dmin[j];
        *dk = dmin[j];
    }

    // Neighbour update with probability 1/T: record the channels that fired.
    const U32x4 w1 = philox4x32_10((uint32_t)p, a.t, 1u, 0u, a.c.key0, a.c.key1);
    uint32_t fire = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!active[j] || F[j]) continue;
        const uint32_t a1 = w1.v[j];
        if ((float)(a1 >> 16) * inv16 * T[j] < 1.0f) {
            const int d = (int)((a1 >> 13) & 7u);
            const int nx = x + nb_dx(d), ny = y + nb_dy(d);
            if (nx >= 0 && nx < a.W && ny >= 0 && ny < a.H) fire |= 1u << j;
        }
    }

    // Decision threshold and update rate (d_bar from the float sum).
    const float rdn = 1.0f - a.c.R_incdec, rup = 1.0f + a.c.R_incdec;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!active[j]) continue;
        const float dbar = S[j] / (float)N;
        const float r = (R[j] > dbar * a.c.R_scale) ? R[j] * rdn : R[j] * rup;
        R[j] = fmaxf(r, a.c.R_lower[j]);
        const float q = (F[j] ? a.c.T_inc : a.c.T_dec) / dbar;
        const float tt = F[j] ? T[j] + q : T[j] - q;
        T[j] = fminf(fmaxf(tt, a.c.T_lower), a.c.T_upper);
    }
    a.m.R[p] = make_float4(R[0], R[1], R[2], R[3]);
    a.m.T[p] = make_float4(T[0], T[1], T[2], T[3]);
    a.m.S[p] = make_float4(S[0], S[1], S[2], S[3]);
    a.m.last[p] = Iw;
    a.m.last_g[p] = Mw;
    a.m.fire[a.t & 1u][p] = (uint8_t)fire;
}

// The neighbour writes of the last processed frame applied for a state read-out (as
// the plain variant's flush, writing the value and the colour magnitudes).
__global__ __launch_bounds__(256) void pbas_grad_flush_kernel(PbasGradPlanes m, int H, int W, uint32_t t_prev,
                                                              int N, uint32_t k0, uint32_t k1) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= H * W) return;
    const int y = p / W, x = p - y * W;
    const int64_t npix = (int64_t)H * W;
    const uint32_t lastw = m.last[p], lastg = m.last_g[p];
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
            const int64_t o = (int64_t)slot * npix + p;
            reinterpret_cast<uint8_t*>(m.samples + o)[j] = (uint8_t)val;
            if (j < 3) reinterpret_cast<uint8_t*>(m.gsamples + o)[j] = (uint8_t)(lastg >> (8 * j));
        }
    }
}

__global__ void pbas_grad_init_kernel(PbasGradPlanes m, int npix, float4 Rl, float Tl) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    m.R[p] = Rl;
    m.T[p] = make_float4(Tl, Tl, Tl, Tl);
}

// Canonical planes: D [N][4] float32, R, T, S [4] float32 <-> float4 per pixel.
__global__ void pbas_grad_export_kernel(PbasGradPlanes m, int npix, int N, float* dout, float* rts) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    for (int k = 0; k < N; ++k) {
        const float4 d = m.D[(int64_t)k * n + p];
        dout[(4 * k + 0) * n + p] = d.x;
        dout[(4 * k + 1) * n + p] = d.y;
        dout[(4 * k + 2) * n + p] = d.z;
        dout[(4 * k + 3) * n + p] = d.w;
    }
    const float4 r = m.R[p], t = m.T[p], s = m.S[p];
    const float v[12] = {r.x, r.y, r.z, r.w, t.x, t.y, t.z, t.w, s.x, s.y, s.z, s.w};
    for (int i = 0; i < 12; ++i) rts[i * n + p] = v[i];
}

__global__ void pbas_grad_import_kernel(PbasGradPlanes m, int npix, int N, const float* din, const float* rts) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    for (int k = 0; k < N; ++k)
        m.D[(int64_t)k * n + p] = make_float4(din[(4 * k + 0) * n + p], din[(4 * k + 1) * n + p],
                                              din[(4 * k + 2) * n + p], din[(4 * k + 3) * n + p]);
    m.R[p] = make_float4(rts[0 * n + p], rts[1 * n + p], rts[2 * n + p], rts[3 * n + p]);
    m.T[p] = make_float4(rts[4 * n + p], rts[5 * n + p], rts[6 * n + p], rts[7 * n + p]);
    m.S[p] = make_float4(rts[8 * n + p], rts[9 * n + p], rts[10 * n + p], rts[11 * n + p]);
}

// The last pushed frame's sums <-> slot (t - 1) mod 3; the other two slots cleared.
// The payload's sums are moved as 32-bit halves (a caller's buffer is 4-byte aligned).
__global__ void pbas_grad_sums_kernel(unsigned long long* gsum, uint32_t* canon, int64_t t, int to_canon) {
    const int j = threadIdx.x;  // 0..2
    const int prev = (int)((t + 2) % 3);
    if (to_canon) {
        const unsigned long long v = t > 0 ? gsum[4 * prev + j] : 0ull;
        canon[2 * j] = (uint32_t)v;
        canon[2 * j + 1] = (uint32_t)(v >> 32);
        return;
    }
    const unsigned long long v = (unsigned long long)canon[2 * j] | ((unsigned long long)canon[2 * j + 1] << 32);
    for (int s = 0; s < 3; ++s) gsum[4 * s + j] = s == prev && t > 0 ? v : 0ull;
}

inline unsigned blocks1d(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t pbas_grad_launch_init_state(const PbasGradPlanes& m, int npix, const PbasConsts& c, hipStream_t s) {
    hipLaunchKernelGGL(pbas_grad_init_kernel, dim3(blocks1d(npix)), dim3(256), 0, s, m, npix,
                       make_float4(c.R_lower[0], c.R_lower[1], c.R_lower[2], c.R_lower[3]), c.T_lower);
    return hipGetLastError();
}

hipError_t pbas_grad_launch_step(const PbasGradArgs& a, hipStream_t s) {
    if ((int64_t)a.t < a.c.N) {
        hipLaunchKernelGGL(pbas_grad_fill_kernel, dim3(blocks1d(a.npix)), dim3(kBlock), 0, s, a);
    } else {
        const int64_t tiles = (int64_t)((a.W + kTileW - 1) / kTileW) * ((a.H + kTileH - 1) / kTileH);
        if (tiles > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(pbas_grad_step_kernel, dim3((unsigned)tiles), dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t pbas_grad_launch_flush(const PbasGradPlanes& m, int H, int W, uint32_t t_prev, const PbasConsts& c,
                                  hipStream_t s) {
    hipLaunchKernelGGL(pbas_grad_flush_kernel, dim3(blocks1d((int64_t)H * W)), dim3(256), 0, s, m, H, W, t_prev,
                       c.N, c.key0, c.key1);
    return hipGetLastError();
}

hipError_t pbas_grad_launch_export(const PbasGradPlanes& m, int npix, int N, int64_t t, uint8_t* out,
                                   hipStream_t s) {
    const size_t plane = (size_t)npix * 4;
    hipError_t e = hipMemcpyAsync(out, m.samples, plane * N, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out + plane * N, m.gsamples, plane * N, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    float* dout = reinterpret_cast<float*>(out + 2 * plane * N);
    float* rts = reinterpret_cast<float*>(out + 6 * plane * N);
    hipLaunchKernelGGL(pbas_grad_export_kernel, dim3(blocks1d(npix)), dim3(256), 0, s, m, npix, N, dout, rts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* canon = reinterpret_cast<uint32_t*>(out + 6 * plane * N + 12 * plane);
    hipLaunchKernelGGL(pbas_grad_sums_kernel, dim3(1), dim3(3), 0, s, m.gsum, canon, t, 1);
    return hipGetLastError();
}

hipError_t pbas_grad_launch_import(const PbasGradPlanes& m, int npix, int N, int64_t t, const uint8_t* in,
                                   hipStream_t s) {
    const size_t plane = (size_t)npix * 4;
    hipError_t e = hipMemcpyAsync(m.samples, in, plane * N, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(m.gsamples, in + plane * N, plane * N, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    const float* din = reinterpret_cast<const float*>(in + 2 * plane * N);
    const float* rts = reinterpret_cast<const float*>(in + 6 * plane * N);
    hipLaunchKernelGGL(pbas_grad_import_kernel, dim3(blocks1d(npix)), dim3(256), 0, s, m, npix, N, din, rts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint32_t* canon = const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(in + 6 * plane * N + 12 * plane));
    hipLaunchKernelGGL(pbas_grad_sums_kernel, dim3(1), dim3(3), 0, s, m.gsum, canon, t, 0);
    return hipGetLastError();
}

}  // namespace fgs
