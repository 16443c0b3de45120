// The per-pixel step of one Gaussian mixture (colour: C = 3 channels, depth:
// C = 1), shared by the plain per-frame kernel and the adjoint window kernels so
// that both run the same IEEE binary32 operations in the same order (Sec. 3.1 and
// the Stauffer-Grimson recursion it builds on).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "fgs_internal.h"

namespace fgs {

template <int K, int C>
struct Mix {
    float w[K];
    float mu[K][C];
    float v[K];
};

// The discrete choices of one step, recorded for the adjoint: the Gaussian that
// attains delta, the matched Gaussian (-1: replacement), whether the variance floor
// applied, and the ranking (3 bits per rank: the pre-ranking index now at that rank).
struct MixRec {
    int argmin;
    int kstar;
    bool clamp;
    uint32_t perm;
};

// Classify on the pre-update mixture (used, delta) and, if `active`, update it in
// place.  With REC, also fill *rec.
template <int K, int C, bool REC>
__device__ __forceinline__ void mixture_step(Mix<K, C>& m, const float (&X)[C], bool active,
                                             float alpha, float lam2, float T_bg, float w_init,
                                             float v_init, float v_min, bool& used,
                                             float& delta, MixRec* rec, bool rho_over_w = false) {
    float q[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float e = X[0] - m.mu[k][0];
        float d2 = e * e;
#pragma unroll
        for (int c = 1; c < C; ++c) {
            e = X[c] - m.mu[k][c];
            d2 = d2 + e * e;
        }
        q[k] = d2 / m.v[k];
    }

    used = m.w[0] > 0.0f;
    int nused = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) nused += (m.w[k] > 0.0f) ? 1 : 0;
    int B = nused;
    bool found = false;
    float cum = 0.0f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        cum = cum + m.w[k];
        if (!found && cum > T_bg) {
            B = k + 1;
            found = true;
        }
    }
    // delta = min over the background Gaussians; the first index attaining it
    delta = q[0];
    int amin = 0;
#pragma unroll
    for (int k = 1; k < K; ++k)
        if (k < B && q[k] < delta) {
            delta = q[k];
            amin = k;
        }
    if (REC) {
        rec->argmin = amin;
        rec->kstar = -1;
        rec->clamp = false;
        uint32_t id = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) id |= (uint32_t)k << (3 * k);
        rec->perm = id;
    }

    if (!active) return;

    int ks = -1;
#pragma unroll
    for (int k = K - 1; k >= 0; --k)
        if (m.w[k] > 0.0f && q[k] < lam2) ks = k;

    const float a = 1.0f - alpha;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float wk = a * m.w[k];
        if (k == ks) wk = wk + alpha;
        m.w[k] = wk;
    }
    if (ks >= 0) {
        // rate of the matched mean and variance: alpha, or alpha over the matched
        // weight just updated (>= alpha > 0)
        float rho = alpha;
        if (rho_over_w) {
            float wm = m.w[0];
#pragma unroll
            for (int k = 1; k < K; ++k)
                if (k == ks) wm = m.w[k];
            rho = alpha / wm;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k != ks) continue;
            float mn[C];
#pragma unroll
            for (int c = 0; c < C; ++c) mn[c] = m.mu[k][c] + rho * (X[c] - m.mu[k][c]);
            float e = X[0] - mn[0];
            float d2 = e * e;
#pragma unroll
            for (int c = 1; c < C; ++c) {
                e = X[c] - mn[c];
                d2 = d2 + e * e;
            }
            float vn = m.v[k] + rho * (d2 - m.v[k]);
            if (REC) rec->clamp = vn < v_min;
            vn = fmaxf(vn, v_min);
#pragma unroll
            for (int c = 0; c < C; ++c) m.mu[k][c] = mn[c];
            m.v[k] = vn;
        }
    } else {
        m.w[K - 1] = w_init;
#pragma unroll
        for (int c = 0; c < C; ++c) m.mu[K - 1][c] = X[c];
        m.v[K - 1] = v_init;
    }

    float S = m.w[0];
#pragma unroll
    for (int k = 1; k < K; ++k) S = S + m.w[k];
#pragma unroll
    for (int k = 0; k < K; ++k) m.w[k] = m.w[k] / S;

    // Rank: insertion network of adjacent compare-exchanges, strictly-greater
    // swaps only, so equal keys keep their order (stable).
    if (REC) rec->kstar = ks;
    float key[K];
    int idx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        key[k] = m.w[k] / sqrtf(m.v[k]);
        idx[k] = k;
    }
    // The network swaps nothing unless some adjacent pair is out of order, which in a
    // static scene is rare: skip it when no lane of the wavefront needs a swap.
    bool unsorted = false;
#pragma unroll
    for (int k = 1; k < K; ++k) unsorted = unsorted || key[k] > key[k - 1];
    if (__any(unsorted))
#pragma unroll
    for (int i = 1; i < K; ++i) {
#pragma unroll
        for (int j = i; j > 0; --j) {
            const bool sw = key[j] > key[j - 1];
            float t;
#define FGS_CSWAP(A, B)      \
    t = sw ? (A) : (B);      \
    (A) = sw ? (B) : (A);    \
    (B) = t;
            FGS_CSWAP(key[j], key[j - 1]);
            {
                const int ti = sw ? idx[j] : idx[j - 1];
                idx[j] = sw ? idx[j - 1] : idx[j];
                idx[j - 1] = ti;
            }
            FGS_CSWAP(m.w[j], m.w[j - 1]);
            FGS_CSWAP(m.v[j], m.v[j - 1]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                FGS_CSWAP(m.mu[j][c], m.mu[j - 1][c]);
            }
#undef FGS_CSWAP
        }
    }
    if (REC) {
        uint32_t pr = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) pr |= (uint32_t)idx[k] << (3 * k);
        rec->perm = pr;
    }
}

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

// One pixel of one frame: ingest, both mixtures' classify-and-update, the
// combined decision, the mask, and the state write-back.  RW selects the rate of
// the matched mean and variance: 0 alpha, 1 alpha / w, 2 as a.c.rho_over_w says
// (a compile-time choice keeps the other path's registers out of the kernel).
template <int KC, int KD, bool NT, int RW = 2>
__device__ __forceinline__ void gmm_pixel(const GmmStepArgs& a, int p) {
    constexpr int E = (KC + 3 * KD + 3) / 4;
    const int y = p / a.W;
    const int x = p - y * a.W;

    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = load_depth(a.depth, a.depth_stride, x, y, a.W, a.H, a.depth_w, a.depth_h);
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
    const bool rw = RW == 2 ? a.c.rho_over_w != 0 : RW == 1;
    mixture_step<KC, 3, false>(mc, Xc, true, a.c.alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_c,
                               a.c.v_min_c, used_c, dc, nullptr, rw);
    mixture_step<KD, 1, false>(md, Xd, valid, a.c.alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_d,
                               a.c.v_min_d, used_d, dd, nullptr, rw);

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

}  // namespace fgs
