// RGB-D Gaussian mixture background model: one fused classify-and-update kernel
// per frame (Sec. 3.1).  One lane per pixel; the pixel's whole state (both
// mixtures) is read once and written once per frame with 16-byte accesses, and
// everything in between stays in registers.  No contraction anywhere: the path
// is a streaming state update bound by HBM bandwidth.
//
// Arithmetic is IEEE binary32, each operation rounded on its own (the library is
// built with -ffp-contract=off; division and square root are correctly rounded),
// in the order of the method:
//   q_k = d2_k / v_k,  d2 = ((e0*e0) + e1*e1) + e2*e2
//   decision on the ranked pre-update mixture: B = leading Gaussians whose
//     weights first sum past T_bg (else those with w > 0), delta = min_{k<B} q_k,
//     Z = (delta_c - lambda^2) + w_d*(delta_d - lambda^2), depth term only where
//     D > 0 and the depth mixture has data; foreground iff Z >= 0
//   update (colour always, depth where D > 0): first k with w_k > 0 and
//     q_k < lambda^2 matches; w = (1-alpha) w (+ alpha if matched); matched
//     mu += alpha (X - mu); v += alpha (|X - mu_new|^2 - v); v >= v_min; no match:
//     Gaussian K-1 = (w_init, X, v_init); w /= sum(w); stable sort by w/sqrt(v).
#include <cstring>

#include "device_common.h"
#include "fgs_internal.h"
#include "gmm_device.h"

namespace fgs {

namespace {

// 512 lanes per workgroup: measured on the 8-model 720p step, GMM K=5 per launch 308.2 us
// with 256 lanes, 302.2 with 512, 313.8 with 1024, 320.9 with 128 (same registers and
// occupancy; larger workgroups retire in fewer, larger pieces, up to the point where one
// no longer fits beside another on a CU).
constexpr int kBlock = 512;

// GEN = false: the default rate and decision compiled in; GEN = true: both read
// from the constants (any other choice).  CV = 3: per-channel colour variances.
// One launch steps b.n models (one for a single push): workgroup w takes pixels
// 256 (w - first[i]) .. +255 of model i, first[i] <= w < first[i + 1].
template <int NB, int KC, int KD, bool NT, bool GEN, int CV>
__global__ __launch_bounds__(kBlock) void gmm_step_kernel(GmmBatch<NB> b) {
    const int w = (int)blockIdx.x;
    int i = 0;
#pragma unroll
    for (int j = 1; j < NB; ++j) i += (j < b.n && w >= b.first[j]) ? 1 : 0;
    const GmmStepArgs& a = b.a[i];
    const int p = (w - b.first[i]) * kBlock + (int)threadIdx.x;
    if (p < a.npix) gmm_pixel<KC, KD, NT, GEN ? 2 : 0, GEN ? 2 : 0, CV>(a, p);
}

// Run-time Kc, Kd indices of the extra-plane fields (fgs_internal.h).
__device__ __forceinline__ int x_wc(int Kc, int Kd, int k) { return gmm_x_wc(Kc, Kd, k); }
__device__ __forceinline__ int x_wd(int Kc, int Kd, int k) { return gmm_x_wd(Kc, Kd, k); }
__device__ __forceinline__ int x_mud(int Kc, int Kd, int k) { return gmm_x_mud(Kc, Kd, k); }
__device__ __forceinline__ int x_vd(int Kc, int Kd, int k) { return gmm_x_vd(Kc, Kd, k); }
__device__ __forceinline__ int x_vg(int Kc, int Kd, int k) { return gmm_x_vg(Kc, Kd, k); }
__device__ __forceinline__ int x_vb(int Kc, int Kd, int k) { return gmm_x_vb(Kc, Kd, k); }

__device__ __forceinline__ float* f4(float4* s, int64_t i) { return reinterpret_cast<float*>(s + i); }
__device__ __forceinline__ const float* f4(const float4* s, int64_t i) {
    return reinterpret_cast<const float*>(s + i);
}
__device__ __forceinline__ float* xf(float4* s, int Kc, int64_t n, int64_t p, int idx) {
    return f4(s, (int64_t)(Kc + idx / 4) * n + p) + idx % 4;
}
__device__ __forceinline__ float xg(const float4* s, int Kc, int64_t n, int64_t p, int idx) {
    return f4(s, (int64_t)(Kc + idx / 4) * n + p)[idx % 4];
}

// Fresh model: w = 0, mu = 0, v = v_init (both mixtures; every colour channel's
// variance when they are per channel).
__global__ void gmm_init_kernel(float4* state, int Kc, int Kd, int var_mode, int npix, float v_init_c,
                                float v_init_d) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    const int E = gmm_extra_planes(Kc, Kd, var_mode);
    for (int k = 0; k < Kc; ++k) state[(int64_t)k * n + p] = make_float4(0.f, 0.f, 0.f, v_init_c);
    for (int e = 0; e < E; ++e) state[(int64_t)(Kc + e) * n + p] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = 0; k < Kd; ++k) *xf(state, Kc, n, p, x_vd(Kc, Kd, k)) = v_init_d;
    if (var_mode)
        for (int k = 0; k < Kc; ++k) {
            *xf(state, Kc, n, p, x_vg(Kc, Kd, k)) = v_init_c;
            *xf(state, Kc, n, p, x_vb(Kc, Kd, k)) = v_init_c;
        }
}

// Canonical order: w_c[Kc], mu_c[Kc][3], v_c[Kc] (per-channel: v_c[Kc][3]), w_d[Kd],
// mu_d[Kd], v_d[Kd], planes of npix.
__global__ void gmm_export_kernel(const float4* state, float* out, int Kc, int Kd, int var_mode, int npix) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    const int nv = var_mode ? 3 : 1;
    for (int k = 0; k < Kc; ++k) {
        const float* c = f4(state, (int64_t)k * n + p);
        out[(int64_t)k * n + p] = xg(state, Kc, n, p, x_wc(Kc, Kd, k));
        for (int ch = 0; ch < 3; ++ch) out[(int64_t)(Kc + 3 * k + ch) * n + p] = c[ch];
        out[(int64_t)(4 * Kc + nv * k) * n + p] = c[3];
        if (var_mode) {
            out[(int64_t)(4 * Kc + nv * k + 1) * n + p] = xg(state, Kc, n, p, x_vg(Kc, Kd, k));
            out[(int64_t)(4 * Kc + nv * k + 2) * n + p] = xg(state, Kc, n, p, x_vb(Kc, Kd, k));
        }
    }
    const int d0 = (4 + nv) * Kc;
    for (int k = 0; k < Kd; ++k) {
        out[(int64_t)(d0 + k) * n + p] = xg(state, Kc, n, p, x_wd(Kc, Kd, k));
        out[(int64_t)(d0 + Kd + k) * n + p] = xg(state, Kc, n, p, x_mud(Kc, Kd, k));
        out[(int64_t)(d0 + 2 * Kd + k) * n + p] = xg(state, Kc, n, p, x_vd(Kc, Kd, k));
    }
}

__global__ void gmm_import_kernel(float4* state, const float* in, int Kc, int Kd, int var_mode, int npix) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    const int E = gmm_extra_planes(Kc, Kd, var_mode);
    const int nv = var_mode ? 3 : 1;
    for (int e = 0; e < E; ++e) state[(int64_t)(Kc + e) * n + p] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = 0; k < Kc; ++k) {
        float* c = f4(state, (int64_t)k * n + p);
        for (int ch = 0; ch < 3; ++ch) c[ch] = in[(int64_t)(Kc + 3 * k + ch) * n + p];
        c[3] = in[(int64_t)(4 * Kc + nv * k) * n + p];
        *xf(state, Kc, n, p, x_wc(Kc, Kd, k)) = in[(int64_t)k * n + p];
        if (var_mode) {
            *xf(state, Kc, n, p, x_vg(Kc, Kd, k)) = in[(int64_t)(4 * Kc + nv * k + 1) * n + p];
            *xf(state, Kc, n, p, x_vb(Kc, Kd, k)) = in[(int64_t)(4 * Kc + nv * k + 2) * n + p];
        }
    }
    const int d0 = (4 + nv) * Kc;
    for (int k = 0; k < Kd; ++k) {
        *xf(state, Kc, n, p, x_wd(Kc, Kd, k)) = in[(int64_t)(d0 + k) * n + p];
        *xf(state, Kc, n, p, x_mud(Kc, Kd, k)) = in[(int64_t)(d0 + Kd + k) * n + p];
        *xf(state, Kc, n, p, x_vd(Kc, Kd, k)) = in[(int64_t)(d0 + 2 * Kd + k) * n + p];
    }
}

template <int NB, int KC, int KD, bool GEN, int CV>
void launch_step_g(const GmmBatch<NB>& b, unsigned grid, hipStream_t s) {
    if (b.a[0].streaming)
        hipLaunchKernelGGL((gmm_step_kernel<NB, KC, KD, true, GEN, CV>), dim3(grid), dim3(kBlock), 0, s, b);
    else
        hipLaunchKernelGGL((gmm_step_kernel<NB, KC, KD, false, GEN, CV>), dim3(grid), dim3(kBlock), 0, s, b);
}

// Kernel variant of a model's constants: 2 per-channel variances, 1 rate or decision
// variant, 0 the defaults compiled in.
int variant(const GmmConsts& c) { return c.var_mode ? 2 : ((c.rho_mode || c.decision) ? 1 : 0); }

template <int NB, int KC, int KD>
hipError_t launch_step_t(const GmmBatch<NB>& b, unsigned grid, hipStream_t s) {
    switch (variant(b.a[0].c)) {
        case 2: launch_step_g<NB, KC, KD, true, 3>(b, grid, s); break;
        case 1: launch_step_g<NB, KC, KD, true, 1>(b, grid, s); break;
        default: launch_step_g<NB, KC, KD, false, 1>(b, grid, s); break;
    }
    return hipGetLastError();
}

template <int NB>
hipError_t launch_batch(const GmmStepArgs* a, int n, int Kc, int Kd, hipStream_t s) {
    GmmBatch<NB> b;
    std::memset(&b, 0, sizeof b);
    b.n = n;
    int64_t grid = 0;
    for (int i = 0; i < n; ++i) {
        b.a[i] = a[i];
        b.first[i] = (int32_t)grid;
        grid += (a[i].npix + kBlock - 1) / kBlock;
    }
    for (int i = n; i <= NB; ++i) b.first[i] = (int32_t)grid;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const unsigned g = (unsigned)grid;
    switch (Kc * 8 + Kd) {
        case 1 * 8 + 1: return launch_step_t<NB, 1, 1>(b, g, s);
        case 2 * 8 + 2: return launch_step_t<NB, 2, 2>(b, g, s);
        case 3 * 8 + 3: return launch_step_t<NB, 3, 3>(b, g, s);
        case 4 * 8 + 4: return launch_step_t<NB, 4, 4>(b, g, s);
        case 5 * 8 + 5: return launch_step_t<NB, 5, 5>(b, g, s);
        case 6 * 8 + 6: return launch_step_t<NB, 6, 6>(b, g, s);
        case 7 * 8 + 7: return launch_step_t<NB, 7, 7>(b, g, s);
        case 7 * 8 + 3: return launch_step_t<NB, 7, 3>(b, g, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool gmm_supported(int Kc, int Kd) {
    if (Kc == Kd && Kc >= 1 && Kc <= 7) return true;
    return Kc == 7 && Kd == 3;
}

int gmm_batch_key(const GmmStepArgs& a, int Kc, int Kd) {
    return ((Kc * 8 + Kd) * 4 + variant(a.c)) * 2 + (a.streaming ? 1 : 0);
}

hipError_t gmm_launch_step_batch(const GmmStepArgs* a, int n, int Kc, int Kd, hipStream_t s) {
    if (n < 1 || n > kBatchMax) return hipErrorInvalidValue;
    for (int i = 1; i < n; ++i)
        if (gmm_batch_key(a[i], Kc, Kd) != gmm_batch_key(a[0], Kc, Kd)) return hipErrorInvalidValue;
    return n == 1 ? launch_batch<1>(a, n, Kc, Kd, s) : launch_batch<kBatchMax>(a, n, Kc, Kd, s);
}

hipError_t gmm_launch_step(const GmmStepArgs& a, int Kc, int Kd, hipStream_t s) {
    return gmm_launch_step_batch(&a, 1, Kc, Kd, s);
}

hipError_t gmm_launch_init(float4* state, int Kc, int Kd, int npix, const GmmConsts& c,
                           hipStream_t s) {
    const unsigned grid = (unsigned)((npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(gmm_init_kernel, dim3(grid), dim3(kBlock), 0, s, state, Kc, Kd, c.var_mode, npix,
                       c.v_init_c, c.v_init_d);
    return hipGetLastError();
}

hipError_t gmm_launch_export(const float4* state, float* out, int Kc, int Kd, int var_mode, int npix,
                             hipStream_t s) {
    const unsigned grid = (unsigned)((npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(gmm_export_kernel, dim3(grid), dim3(kBlock), 0, s, state, out, Kc, Kd, var_mode, npix);
    return hipGetLastError();
}

hipError_t gmm_launch_import(float4* state, const float* in, int Kc, int Kd, int var_mode, int npix,
                             hipStream_t s) {
    const unsigned grid = (unsigned)((npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(gmm_import_kernel, dim3(grid), dim3(kBlock), 0, s, state, in, Kc, Kd, var_mode, npix);
    return hipGetLastError();
}

}  // namespace fgs
