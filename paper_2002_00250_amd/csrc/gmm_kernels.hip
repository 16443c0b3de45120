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
#include "device_common.h"
#include "fgs_internal.h"
#include "gmm_device.h"

namespace fgs {

namespace {

constexpr int kBlock = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));
// State planes are touched once per frame.  When the device's resident model
// state exceeds the last-level (Infinity) cache the kernels stream it with
// non-temporal loads and stores; otherwise ordinary accesses let a cache-sized
// working set stay resident between frames.
template <bool NT>
__device__ __forceinline__ float4 ld_state(const float4* p) {
    if constexpr (NT) {
        const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ void st_state(float4* p, float4 v) {
    if constexpr (NT) {
        f32x4 w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<f32x4*>(p));
    } else {
        *p = v;
    }
}

template <int KC, int KD, bool NT>
__global__ __launch_bounds__(kBlock) void gmm_step_kernel(GmmStepArgs a) {
    constexpr int E = (KC + 3 * KD + 3) / 4;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.npix) return;
    const int y = p / a.W;
    const int x = p - y * a.W;

    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = *reinterpret_cast<const uint16_t*>(a.depth + (int64_t)y * a.depth_stride + 2 * x);
    const float Xc[3] = {(float)px[0], (float)px[1], (float)px[2]};
    const bool valid = dmm > 0u;
    const float Xd[1] = {(float)depth_code(dmm, a.c.depth_max_mm)};

    const float4* st = a.state;
    float4 core[KC];
    float ex[4 * E];
#pragma unroll
    for (int k = 0; k < KC; ++k) core[k] = ld_state<NT>(st + (int64_t)k * a.npix + p);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const float4 f = ld_state<NT>(st + (int64_t)(KC + e) * a.npix + p);
        ex[4 * e + 0] = f.x;
        ex[4 * e + 1] = f.y;
        ex[4 * e + 2] = f.z;
        ex[4 * e + 3] = f.w;
    }
    Mix<KC, 3> mc;
    Mix<KD, 1> md;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        mc.w[k] = core[k].x;
        mc.mu[k][0] = core[k].y;
        mc.mu[k][1] = core[k].z;
        mc.mu[k][2] = core[k].w;
        mc.v[k] = ex[k];
    }
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        md.w[k] = ex[KC + k];
        md.mu[k][0] = ex[KC + KD + k];
        md.v[k] = ex[KC + 2 * KD + k];
    }

    const float lam2 = a.c.lam * a.c.lam;
    bool used_c, used_d;
    float dc, dd;
    mixture_step<KC, 3, false>(mc, Xc, true, a.c.alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_c,
                        a.c.v_min_c, used_c, dc, nullptr);
    mixture_step<KD, 1, false>(md, Xd, valid, a.c.alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_d,
                        a.c.v_min_d, used_d, dd, nullptr);

    const bool term_c = used_c;
    const bool term_d = valid && used_d;
    const float tc = dc - lam2;
    const float td = a.c.w_depth * (dd - lam2);
    const float Z = term_c ? (term_d ? tc + td : tc) : td;
    a.mask[p] = ((term_c || term_d) && Z >= 0.0f) ? (uint8_t)255 : (uint8_t)0;

    float4* so = a.state;
#pragma unroll
    for (int k = 0; k < KC; ++k)
        st_state<NT>(so + (int64_t)k * a.npix + p, make_float4(mc.w[k], mc.mu[k][0], mc.mu[k][1], mc.mu[k][2]));
#pragma unroll
    for (int k = 0; k < KC; ++k) ex[k] = mc.v[k];
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        ex[KC + k] = md.w[k];
        ex[KC + KD + k] = md.mu[k][0];
        ex[KC + 2 * KD + k] = md.v[k];
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
        st_state<NT>(so + (int64_t)(KC + e) * a.npix + p,
                  make_float4(ex[4 * e + 0], ex[4 * e + 1], ex[4 * e + 2], ex[4 * e + 3]));
}

// Fresh model: w = 0, mu = 0, v = v_init (both mixtures).
__global__ void gmm_init_kernel(float4* state, int Kc, int Kd, int npix, float v_init_c,
                                float v_init_d) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int E = (Kc + 3 * Kd + 3) / 4;
    for (int k = 0; k < Kc; ++k) state[(int64_t)k * npix + p] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int e = 0; e < E; ++e) {
        float f[4];
        for (int i = 0; i < 4; ++i) {
            const int idx = 4 * e + i;
            float val = 0.f;
            if (idx < Kc) val = v_init_c;
            else if (idx >= Kc + 2 * Kd && idx < Kc + 3 * Kd) val = v_init_d;
            f[i] = val;
        }
        state[(int64_t)(Kc + e) * npix + p] = make_float4(f[0], f[1], f[2], f[3]);
    }
}

__device__ __forceinline__ float* f4(float4* s, int64_t i) { return reinterpret_cast<float*>(s + i); }
__device__ __forceinline__ const float* f4(const float4* s, int64_t i) {
    return reinterpret_cast<const float*>(s + i);
}

// Canonical order: w_c[Kc], mu_c[Kc][3], v_c[Kc], w_d[Kd], mu_d[Kd], v_d[Kd], planes of npix.
__global__ void gmm_export_kernel(const float4* state, float* out, int Kc, int Kd, int npix) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    for (int k = 0; k < Kc; ++k) {
        const float* c = f4(state, (int64_t)k * n + p);
        out[(int64_t)k * n + p] = c[0];
        for (int ch = 0; ch < 3; ++ch) out[(int64_t)(Kc + 3 * k + ch) * n + p] = c[1 + ch];
    }
    auto extra = [&](int idx) { return f4(state, (int64_t)(Kc + idx / 4) * n + p)[idx % 4]; };
    for (int k = 0; k < Kc; ++k) out[(int64_t)(4 * Kc + k) * n + p] = extra(k);
    for (int k = 0; k < Kd; ++k) {
        out[(int64_t)(5 * Kc + k) * n + p] = extra(Kc + k);
        out[(int64_t)(5 * Kc + Kd + k) * n + p] = extra(Kc + Kd + k);
        out[(int64_t)(5 * Kc + 2 * Kd + k) * n + p] = extra(Kc + 2 * Kd + k);
    }
}

__global__ void gmm_import_kernel(float4* state, const float* in, int Kc, int Kd, int npix) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int64_t n = npix;
    for (int k = 0; k < Kc; ++k) {
        float* c = f4(state, (int64_t)k * n + p);
        c[0] = in[(int64_t)k * n + p];
        for (int ch = 0; ch < 3; ++ch) c[1 + ch] = in[(int64_t)(Kc + 3 * k + ch) * n + p];
    }
    const int E = (Kc + 3 * Kd + 3) / 4;
    for (int idx = 0; idx < 4 * E; ++idx) {
        float v = 0.f;
        if (idx < Kc) v = in[(int64_t)(4 * Kc + idx) * n + p];
        else if (idx < Kc + Kd) v = in[(int64_t)(5 * Kc + (idx - Kc)) * n + p];
        else if (idx < Kc + 2 * Kd) v = in[(int64_t)(5 * Kc + Kd + (idx - Kc - Kd)) * n + p];
        else if (idx < Kc + 3 * Kd) v = in[(int64_t)(5 * Kc + 2 * Kd + (idx - Kc - 2 * Kd)) * n + p];
        f4(state, (int64_t)(Kc + idx / 4) * n + p)[idx % 4] = v;
    }
}

template <int KC, int KD>
hipError_t launch_step_t(const GmmStepArgs& a, hipStream_t s) {
    const unsigned grid = (unsigned)((a.npix + kBlock - 1) / kBlock);
    if (a.streaming)
        hipLaunchKernelGGL((gmm_step_kernel<KC, KD, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((gmm_step_kernel<KC, KD, false>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace

bool gmm_supported(int Kc, int Kd) {
    if (Kc == Kd && Kc >= 1 && Kc <= 7) return true;
    return Kc == 7 && Kd == 3;
}

hipError_t gmm_launch_step(const GmmStepArgs& a, int Kc, int Kd, hipStream_t s) {
    switch (Kc * 8 + Kd) {
        case 1 * 8 + 1: return launch_step_t<1, 1>(a, s);
        case 2 * 8 + 2: return launch_step_t<2, 2>(a, s);
        case 3 * 8 + 3: return launch_step_t<3, 3>(a, s);
        case 4 * 8 + 4: return launch_step_t<4, 4>(a, s);
        case 5 * 8 + 5: return launch_step_t<5, 5>(a, s);
        case 6 * 8 + 6: return launch_step_t<6, 6>(a, s);
        case 7 * 8 + 7: return launch_step_t<7, 7>(a, s);
        case 7 * 8 + 3: return launch_step_t<7, 3>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t gmm_launch_init(float4* state, int Kc, int Kd, int npix, const GmmConsts& c,
                           hipStream_t s) {
    const unsigned grid = (unsigned)((npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(gmm_init_kernel, dim3(grid), dim3(kBlock), 0, s, state, Kc, Kd, npix,
                       c.v_init_c, c.v_init_d);
    return hipGetLastError();
}

hipError_t gmm_launch_export(const float4* state, float* out, int Kc, int Kd, int npix,
                             hipStream_t s) {
    const unsigned grid = (unsigned)((npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(gmm_export_kernel, dim3(grid), dim3(kBlock), 0, s, state, out, Kc, Kd, npix);
    return hipGetLastError();
}

hipError_t gmm_launch_import(float4* state, const float* in, int Kc, int Kd, int npix,
                             hipStream_t s) {
    const unsigned grid = (unsigned)((npix + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(gmm_import_kernel, dim3(grid), dim3(kBlock), 0, s, state, in, Kc, Kd, npix);
    return hipGetLastError();
}

}  // namespace fgs
