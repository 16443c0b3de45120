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

// One mixture: K Gaussians over C channels.  CV = 1: one variance per Gaussian (v);
// CV = 3: one per channel, channel 0 in v and channels 1, 2 in vx.
template <int K, int C, int CV = 1>
struct Mix {
    float w[K];
    float mu[K][C];
    float v[K];
    float vx[K][CV == 3 ? 2 : 1];
};

// The single variance of Gaussian k: v, or the sum of the per-channel variances.
template <int K, int C, int CV>
__device__ __forceinline__ float var_sum(const Mix<K, C, CV>& m, int k) {
    if constexpr (CV == 3) return (m.v[k] + m.vx[k][0]) + m.vx[k][1];
    else return m.v[k];
}

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
// With `chg`, also report which ranks may hold a different (mean, variance) than
// before the step: bit r is set when the ranking moved another Gaussian to rank r
// or when the Gaussian at rank r was matched or replaced (clear bits are certain).
// With `vsel`, also the (pre-update) variance of the Gaussian attaining delta.
template <int K, int C, bool REC, int CV = 1>
__device__ __forceinline__ void mixture_step(Mix<K, C, CV>& m, const float (&X)[C], bool active,
                                             float alpha, float lam2, float T_bg, float w_init,
                                             float v_init, float v_min, bool& used,
                                             float& delta, MixRec* rec, int rho_mode = 0,
                                             uint32_t* chg = nullptr, float* vsel = nullptr) {
    if (chg) *chg = 0u;
    float q[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if constexpr (CV == 3) {  // squared Mahalanobis distance, diagonal covariance
            float e = X[0] - m.mu[k][0];
            float acc = (e * e) / m.v[k];
            e = X[1] - m.mu[k][1];
            acc = acc + (e * e) / m.vx[k][0];
            e = X[2] - m.mu[k][2];
            acc = acc + (e * e) / m.vx[k][1];
            q[k] = acc;
        } else {
            float e = X[0] - m.mu[k][0];
            float d2 = e * e;
#pragma unroll
            for (int c = 1; c < C; ++c) {
                e = X[c] - m.mu[k][c];
                d2 = d2 + e * e;
            }
            q[k] = d2 / m.v[k];
        }
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
    if (vsel) {
        float vs = var_sum(m, 0);
#pragma unroll
        for (int k = 1; k < K; ++k)
            if (k == amin) vs = var_sum(m, k);
        *vsel = vs;
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
        // rate of the matched mean and variance: alpha; alpha over the matched weight
        // just updated (>= alpha > 0); or alpha times the Eq. (1) density of the
        // matched Gaussian at the sample, before its update
        float rho = alpha;
        if (rho_mode != 0) {
            float wm = m.w[0], qm = q[0], vm = var_sum(m, 0);
#pragma unroll
            for (int k = 1; k < K; ++k)
                if (k == ks) {
                    wm = m.w[k];
                    qm = q[k];
                    vm = var_sum(m, k);
                }
            rho = rho_mode == 1 ? alpha / wm : alpha * (expf(-0.5f * qm) / (6.28318530717958647692f * vm));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k != ks) continue;
            float mn[C];
#pragma unroll
            for (int c = 0; c < C; ++c) mn[c] = m.mu[k][c] + rho * (X[c] - m.mu[k][c]);
            if constexpr (CV == 3) {  // each channel's variance on its own deviation and floor
                float e = X[0] - mn[0];
                m.v[k] = fmaxf(m.v[k] + rho * (e * e - m.v[k]), v_min);
                e = X[1] - mn[1];
                m.vx[k][0] = fmaxf(m.vx[k][0] + rho * (e * e - m.vx[k][0]), v_min);
                e = X[2] - mn[2];
                m.vx[k][1] = fmaxf(m.vx[k][1] + rho * (e * e - m.vx[k][1]), v_min);
            } else {
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
                m.v[k] = vn;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) m.mu[k][c] = mn[c];
        }
    } else {
        m.w[K - 1] = w_init;
#pragma unroll
        for (int c = 0; c < C; ++c) m.mu[K - 1][c] = X[c];
        m.v[K - 1] = v_init;
        if constexpr (CV == 3) m.vx[K - 1][0] = m.vx[K - 1][1] = v_init;
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
        key[k] = m.w[k] / sqrtf(var_sum(m, k));
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
            if constexpr (CV == 3) {
                FGS_CSWAP(m.vx[j][0], m.vx[j - 1][0]);
                FGS_CSWAP(m.vx[j][1], m.vx[j - 1][1]);
            }
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
    if (chg) {
        const int touched = ks >= 0 ? ks : K - 1;  // matched, or replaced
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < K; ++r) c |= (uint32_t)(idx[r] != r || idx[r] == touched) << r;
        *chg = c;
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

// Device layout of a GMM model (planes of npix float4, plane-major):
//   core plane k (k < Kc):  (mu_r, mu_g, mu_b, v) of colour rank k (with per-channel
//   colour variances, CV = 3: v is the red one);
//   extra planes (E of them): the floats w_c[0..Kc-1], w_d[0..Kd-1], then
//   (mu_d, v_d) of depth rank 0, 1, ..., then (CV = 3) the (v_g, v_b) of colour
//   rank 0, 1, ..., packed four to a plane, zero padded.
// Weights decay every frame, but a rank's mean and variance change only when its
// Gaussian is matched, replaced or moved by the ranking, so the planes that hold
// only means and variances can often be left unwritten.
template <int KC, int KD, int CV = 1>
struct GmmLayout {
    static constexpr int NX = KC + 3 * KD + (CV == 3 ? 2 * KC : 0);  // extra floats
    static constexpr int E = (NX + 3) / 4;                            // extra planes
    static constexpr int w_c(int k) { return gmm_x_wc(KC, KD, k); }
    static constexpr int w_d(int k) { return gmm_x_wd(KC, KD, k); }
    static constexpr int mu_d(int k) { return gmm_x_mud(KC, KD, k); }
    static constexpr int v_d(int k) { return gmm_x_vd(KC, KD, k); }
    static constexpr int v_g(int k) { return gmm_x_vg(KC, KD, k); }
    static constexpr int v_b(int k) { return gmm_x_vb(KC, KD, k); }
};

// Scaled Eq. (1) factor of the Gaussian attaining delta (decision 1), in the order
// the oracle rounds it: s * (exp(-delta/2) / (2 pi v)).
__device__ __forceinline__ float density_factor(float delta, float v, float s) {
    return s * (expf(-0.5f * delta) / (6.28318530717958647692f * v));
}

// One pixel of one frame: ingest, both mixtures' classify-and-update, the
// combined decision, the mask, and the state write-back.  RW selects the rate of
// the matched mean and variance: 0 alpha, 1 as a.c.rho_mode says;
// DEC the decision: 0 the Z rule, 1 the density product, 2 as a.c.decision says
// (a compile-time choice keeps the other path's registers out of the kernel).
// A plane is stored only where one of the 4 pixels sharing the lane's 64-byte
// sector of it (lanes 4i..4i+3: 16 bytes per pixel) may have changed it, so every
// store still covers whole sectors.
// Bit i of the result: bit i of `bits` set in any of lanes 4i..4i+3 (one plane per bit).
__device__ __forceinline__ uint32_t sector_or(uint32_t bits) {
    bits |= __shfl_xor(bits, 1, 64);
    bits |= __shfl_xor(bits, 2, 64);
    return bits;
}

template <int KC, int KD, bool NT, int RW = 2, int DEC = 2, int CV = 1>
__device__ __forceinline__ void gmm_pixel(const GmmStepArgs& a, int p) {
    using L = GmmLayout<KC, KD, CV>;
    constexpr int E = L::E;
    const int y = p / a.W;
    const int x = p - y * a.W;

    // Every read is issued before any result is used (the frame first, then the
    // state planes): loads complete in order, and the depth code's branch would
    // otherwise wait for the frame before the state reads go out.
    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = load_depth(a.depth, a.depth_stride, x, y, a.W, a.H, a.depth_w, a.depth_h);
    const uint32_t r0 = px[0], r1 = px[1], r2 = px[2];
    const float4* st = a.state;
    float4 core[KC];
    float4 exv[E];
#pragma unroll
    for (int k = 0; k < KC; ++k) core[k] = ld_state<NT>(st + (int64_t)k * a.npix + p);
#pragma unroll
    for (int e = 0; e < E; ++e) exv[e] = ld_state<NT>(st + (int64_t)(KC + e) * a.npix + p);
    __builtin_amdgcn_sched_barrier(0);

    const float Xc[3] = {(float)r0, (float)r1, (float)r2};
    const bool valid = dmm > 0u;
    const float Xd[1] = {(float)depth_code(dmm, a.c.depth_max_mm)};
    float ex[4 * E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        ex[4 * e + 0] = exv[e].x;
        ex[4 * e + 1] = exv[e].y;
        ex[4 * e + 2] = exv[e].z;
        ex[4 * e + 3] = exv[e].w;
    }
    Mix<KC, 3, CV> mc;
    Mix<KD, 1> md;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        mc.w[k] = ex[L::w_c(k)];
        mc.mu[k][0] = core[k].x;
        mc.mu[k][1] = core[k].y;
        mc.mu[k][2] = core[k].z;
        mc.v[k] = core[k].w;
        if constexpr (CV == 3) {
            mc.vx[k][0] = ex[L::v_g(k)];
            mc.vx[k][1] = ex[L::v_b(k)];
        }
    }
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        md.w[k] = ex[L::w_d(k)];
        md.mu[k][0] = ex[L::mu_d(k)];
        md.v[k] = ex[L::v_d(k)];
    }

    const float lam2 = a.c.lam * a.c.lam;
    bool used_c, used_d;
    float dc, dd;
    uint32_t chg_c, chg_d;
    float vsel_c = 1.0f, vsel_d = 1.0f;
    const int rw = RW == 0 ? 0 : a.c.rho_mode;
    const bool dec = DEC == 2 ? a.c.decision != 0 : DEC == 1;
    float4* so = a.state;
    mixture_step<KC, 3, false, CV>(mc, Xc, true, a.c.alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_c,
                               a.c.v_min_c, used_c, dc, nullptr, rw, &chg_c, DEC ? &vsel_c : nullptr);
    // the colour means and variances are final: store them before the depth step
    const uint32_t wc = sector_or(chg_c);
#pragma unroll
    for (int k = 0; k < KC; ++k)
        if ((wc >> k) & 1u)
            st_state<NT>(so + (int64_t)k * a.npix + p, make_float4(mc.mu[k][0], mc.mu[k][1], mc.mu[k][2], mc.v[k]));
    mixture_step<KD, 1, false>(md, Xd, valid, a.c.alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_d,
                               a.c.v_min_d, used_d, dd, nullptr, rw, &chg_d, DEC ? &vsel_d : nullptr);

    const bool term_c = used_c;
    const bool term_d = valid && used_d;
    bool fg;
    if (DEC != 0 && dec) {
        const float Pc = density_factor(dc, vsel_c, a.c.density_scale);
        const float Pd = density_factor(dd, vsel_d, a.c.density_scale);
        const float P = term_c ? (term_d ? Pc * Pd : Pc) : Pd;
        fg = P < a.c.density_threshold;
    } else {
        const float tc = dc - lam2;
        const float td = a.c.w_depth * (dd - lam2);
        const float Z = term_c ? (term_d ? tc + td : tc) : td;
        fg = Z >= 0.0f;
    }
    a.mask[p] = ((term_c || term_d) && fg) ? (uint8_t)255 : (uint8_t)0;

    // Which extra floats may change: the colour weights always (the colour mixture
    // is updated every frame), the depth weights where depth > 0 (the depth mixture
    // is updated only there), a depth mean and variance as the depth mixture reports.
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        ex[L::w_c(k)] = mc.w[k];
        if constexpr (CV == 3) {
            ex[L::v_g(k)] = mc.vx[k][0];
            ex[L::v_b(k)] = mc.vx[k][1];
        }
    }
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        ex[L::w_d(k)] = md.w[k];
        ex[L::mu_d(k)] = md.mu[k][0];
        ex[L::v_d(k)] = md.v[k];
    }
    uint32_t che = 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        bool ch = false;
#pragma unroll
        for (int i = 4 * e; i < 4 * e + 4; ++i) {
            if (i < KC) ch = true;
            else if (i < KC + KD) ch = ch || valid;
            else if (i < KC + 3 * KD) ch = ch || ((chg_d >> ((i - KC - KD) >> 1)) & 1u);
            else if (i < L::NX) ch = ch || ((chg_c >> ((i - KC - 3 * KD) >> 1)) & 1u);
        }
        che |= (ch ? 1u : 0u) << e;
    }
    const uint32_t we = sector_or(che);
#pragma unroll
    for (int e = 0; e < E; ++e)
        if ((we >> e) & 1u)
            st_state<NT>(so + (int64_t)(KC + e) * a.npix + p,
                         make_float4(ex[4 * e + 0], ex[4 * e + 1], ex[4 * e + 2], ex[4 * e + 3]));
}

}  // namespace fgs
