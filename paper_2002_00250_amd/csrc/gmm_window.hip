// Adjoint of the RGB-D GMM recursion over a window of frames.
//
// Parameters theta = (alpha, lambda, w_d), read from device memory.  The window
// starts from a fresh model; every frame yields the pre-update score
//   Z_t = (delta_c - lambda^2) + w_d (delta_d - lambda^2)
// (terms only where the model has data; depth only where D > 0), exactly the
// quantity the plain kernel thresholds at 0 for the mask (Sec. 3.1 reading).
//
// Forward: one lane per pixel runs all T frames with the state in registers,
// writing Z_t, the term flags, a 64-bit record of the step's discrete choices
// (argmin of delta, matched Gaussian or replacement, variance floor, ranking)
// for both mixtures, and a checkpoint of the means and variances every E frames.
//
// Backward: with the recorded choices held fixed the weights reach Z only through
// discrete choices, so their adjoints vanish; alpha's gradient flows through the
// matched Gaussian's mean and variance updates.  Each lane walks the segments in
// reverse: it replays the segment's means/variances from the checkpoint into a
// scratch buffer (same fp32 operations as the forward, so the same values), then
// runs the reverse sweep over the segment.  Per-lane gradients accumulate in
// fp64 and are reduced in a fixed order (block tree, then one block over the
// block partials), so the result is deterministic.
#include "device_common.h"
#include "fgs_internal.h"
#include "gmm_device.h"

namespace fgs {

namespace {

constexpr int kBlock = 256;

// Record layout, per mixture (colour in bits 0..31, depth in 32..63):
//   bit 0 term, bits 1-3 argmin, bit 4 active, bits 5-7 matched (7 = replaced),
//   bit 8 floor applied, bits 9.. ranking (3 bits per rank).
__device__ __forceinline__ uint32_t pack_rec(const MixRec& r, bool term, bool active) {
    return (term ? 1u : 0u) | ((uint32_t)r.argmin << 1) | (active ? 16u : 0u) |
           ((uint32_t)(r.kstar < 0 ? 7 : r.kstar) << 5) | (r.clamp ? 256u : 0u) | (r.perm << 9);
}

// Plane order of the mean/variance snapshots: colour mu[k][c], colour v[k],
// depth mu[k], depth v[k]; F = 6K floats per pixel.
template <int K>
struct MV {
    float muc[K][3], vc[K], mud[K], vd[K];
};

template <int K>
__device__ __forceinline__ void store_mv(const MV<K>& s, float* base, int64_t npix, int p) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) base[(int64_t)(3 * k + c) * npix + p] = s.muc[k][c];
        base[(int64_t)(3 * K + k) * npix + p] = s.vc[k];
        base[(int64_t)(4 * K + k) * npix + p] = s.mud[k];
        base[(int64_t)(5 * K + k) * npix + p] = s.vd[k];
    }
}

template <int K>
__device__ __forceinline__ void load_mv(MV<K>& s, const float* base, int64_t npix, int p) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s.muc[k][c] = base[(int64_t)(3 * k + c) * npix + p];
        s.vc[k] = base[(int64_t)(3 * K + k) * npix + p];
        s.mud[k] = base[(int64_t)(4 * K + k) * npix + p];
        s.vd[k] = base[(int64_t)(5 * K + k) * npix + p];
    }
}

struct Input {
    float Xc[3];
    float Xd[1];
    bool valid;
};

__device__ __forceinline__ Input load_input(const GmmWindowArgs& a, int t, int p) {
    Input in;
    const uint8_t* px = a.rgb + ((int64_t)t * a.npix + p) * 3;
    const uint32_t dmm = a.depth[(int64_t)t * a.npix + p];
    in.Xc[0] = (float)px[0];
    in.Xc[1] = (float)px[1];
    in.Xc[2] = (float)px[2];
    in.valid = dmm > 0u;
    in.Xd[0] = (float)depth_code(dmm, a.c.depth_max_mm);
    return in;
}

template <int K>
__global__ __launch_bounds__(kBlock) void gmm_window_forward_kernel(GmmWindowArgs a) {
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= a.npix) return;
    const float alpha = a.theta[0], lam = a.theta[1], wd = a.theta[2];
    const float lam2 = lam * lam;
    Mix<K, 3> mc;
    Mix<K, 1> md;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        mc.w[k] = 0.f;
        mc.mu[k][0] = mc.mu[k][1] = mc.mu[k][2] = 0.f;
        mc.v[k] = a.c.v_init_c;
        md.w[k] = 0.f;
        md.mu[k][0] = 0.f;
        md.v[k] = a.c.v_init_d;
    }
    const int64_t F = 6 * K;
    for (int t = 0; t < a.T; ++t) {
        if (t % a.E == 0) {
            MV<K> s;
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int c = 0; c < 3; ++c) s.muc[k][c] = mc.mu[k][c];
                s.vc[k] = mc.v[k];
                s.mud[k] = md.mu[k][0];
                s.vd[k] = md.v[k];
            }
            store_mv<K>(s, a.ckpt + (int64_t)(t / a.E) * F * a.npix, a.npix, p);
        }
        const Input in = load_input(a, t, p);
        bool used_c, used_d;
        float dc, dd;
        MixRec rc, rd;
        mixture_step<K, 3, true>(mc, in.Xc, true, alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_c,
                                 a.c.v_min_c, used_c, dc, &rc);
        mixture_step<K, 1, true>(md, in.Xd, in.valid, alpha, lam2, a.c.T_bg, a.c.w_init, a.c.v_init_d,
                                 a.c.v_min_d, used_d, dd, &rd);
        const bool term_c = used_c, term_d = in.valid && used_d;
        const float tc = dc - lam2;
        const float td = wd * (dd - lam2);
        const float Z = term_c ? (term_d ? tc + td : tc) : (term_d ? td : 0.0f);
        const int64_t o = (int64_t)t * a.npix + p;
        a.Z[o] = Z;
        a.has[o] = (term_c || term_d) ? 1 : 0;
        a.rec[o] = (uint64_t)pack_rec(rc, term_c, true) | ((uint64_t)pack_rec(rd, term_d, in.valid) << 32);
    }
}

// Replay of one mixture's means/variances with recorded choices (fp32, the
// forward's operations in the forward's order).
template <int K, int C>
__device__ __forceinline__ void replay_mix(float (&mu)[K][C], float (&v)[K], const float (&X)[C],
                                           uint32_t r, float alpha, float v_init, float v_min) {
    if (!(r & 16u)) return;
    const int ks = (int)((r >> 5) & 7u);
    const bool clamp = (r >> 8) & 1u;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k != ks) continue;
        float mn[C];
#pragma unroll
        for (int c = 0; c < C; ++c) mn[c] = mu[k][c] + alpha * (X[c] - mu[k][c]);
        float e = X[0] - mn[0];
        float d2 = e * e;
#pragma unroll
        for (int c = 1; c < C; ++c) {
            e = X[c] - mn[c];
            d2 = d2 + e * e;
        }
        const float vt = v[k] + alpha * (d2 - v[k]);
#pragma unroll
        for (int c = 0; c < C; ++c) mu[k][c] = mn[c];
        v[k] = clamp ? v_min : vt;
    }
    if (ks == 7) {
#pragma unroll
        for (int c = 0; c < C; ++c) mu[K - 1][c] = X[c];
        v[K - 1] = v_init;
    }
    float nmu[K][C], nv[K];
#pragma unroll
    for (int rk = 0; rk < K; ++rk) {
        const int src = (int)((r >> (9 + 3 * rk)) & 7u);
#pragma unroll
        for (int c = 0; c < C; ++c) nmu[rk][c] = mu[0][c];
        nv[rk] = v[0];
#pragma unroll
        for (int k = 1; k < K; ++k)
            if (src == k) {
#pragma unroll
                for (int c = 0; c < C; ++c) nmu[rk][c] = mu[k][c];
                nv[rk] = v[k];
            }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < C; ++c) mu[k][c] = nmu[k][c];
        v[k] = nv[k];
    }
}

// Adjoint of one mixture's step.  In: pre-step means/variances, the adjoint of the
// post-step means/variances (am, av).  Out: the adjoint of the pre-step values (in
// place) and the step's contribution to d/d alpha.
template <int K, int C>
__device__ __forceinline__ double reverse_mix(const float (&mu)[K][C], const float (&v)[K],
                                              const float (&X)[C], uint32_t r, float alpha,
                                              float (&am)[K][C], float (&av)[K]) {
    if (!(r & 16u)) return 0.0;  // inactive: the state passed through
    // un-rank: post rank rk came from pre index perm(rk)
    float bm[K][C], bv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int c = 0; c < C; ++c) bm[k][c] = 0.f;
        bv[k] = 0.f;
    }
#pragma unroll
    for (int rk = 0; rk < K; ++rk) {
        const int src = (int)((r >> (9 + 3 * rk)) & 7u);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (src == k) {
#pragma unroll
                for (int c = 0; c < C; ++c) bm[k][c] += am[rk][c];
                bv[k] += av[rk];
            }
    }
    const int ks = (int)((r >> 5) & 7u);
    const bool clamp = (r >> 8) & 1u;
    double ga = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k == ks) {
            float mn[C];
#pragma unroll
            for (int c = 0; c < C; ++c) mn[c] = mu[k][c] + alpha * (X[c] - mu[k][c]);
            float d2 = 0.f;
#pragma unroll
            for (int c = 0; c < C; ++c) d2 += (X[c] - mn[c]) * (X[c] - mn[c]);
            const float avt = clamp ? 0.f : bv[k];
            float gam = avt * (d2 - v[k]);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float amn = bm[k][c] + avt * alpha * (-2.0f) * (X[c] - mn[c]);
                gam += amn * (X[c] - mu[k][c]);
                am[k][c] = (1.0f - alpha) * amn;
            }
            av[k] = (1.0f - alpha) * avt;
            ga += (double)gam;
        } else if (ks == 7 && k == K - 1) {
#pragma unroll
            for (int c = 0; c < C; ++c) am[k][c] = 0.f;
            av[k] = 0.f;
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) am[k][c] = bm[k][c];
            av[k] = bv[k];
        }
    }
    return ga;
}

// Z's dependence on the pre-step state through delta = |X - mu_a|^2 / v_a.
template <int K, int C>
__device__ __forceinline__ float score_adjoint(const float (&mu)[K][C], const float (&v)[K],
                                               const float (&X)[C], uint32_t r, float g,
                                               float (&am)[K][C], float (&av)[K]) {
    const int a = (int)((r >> 1) & 7u);
    float delta = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (k != a) continue;
        float e = X[0] - mu[k][0];
        float d2 = e * e;
#pragma unroll
        for (int c = 1; c < C; ++c) {
            e = X[c] - mu[k][c];
            d2 = d2 + e * e;
        }
        delta = d2 / v[k];
#pragma unroll
        for (int c = 0; c < C; ++c) am[k][c] += g * (-2.0f) * (X[c] - mu[k][c]) / v[k];
        av[k] += g * (-delta / v[k]);
    }
    return delta;
}

__device__ __forceinline__ double block_sum(double x, double* sh) {
    sh[threadIdx.x] = x;
    __syncthreads();
#pragma unroll
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int K>
__global__ __launch_bounds__(kBlock) void gmm_window_backward_kernel(GmmWindowArgs a) {
    __shared__ double sh[kBlock];
    const int p = blockIdx.x * kBlock + threadIdx.x;
    double g_alpha = 0.0, g_lam = 0.0, g_wd = 0.0;
    if (p < a.npix) {
        const float alpha = a.theta[0], lam = a.theta[1], wd = a.theta[2];
        const float lam2 = lam * lam;
        const int64_t F = 6 * K;
        float amc[K][3], avc[K], amd[K][1], avd[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            amc[k][0] = amc[k][1] = amc[k][2] = 0.f;
            avc[k] = 0.f;
            amd[k][0] = 0.f;
            avd[k] = 0.f;
        }
        for (int seg = a.nseg - 1; seg >= 0; --seg) {
            const int t0 = seg * a.E;
            const int t1 = min(a.T, t0 + a.E);
            MV<K> s;
            load_mv<K>(s, a.ckpt + (int64_t)seg * F * a.npix, a.npix, p);
            for (int t = t0; t < t1; ++t) {
                store_mv<K>(s, a.scratch + (int64_t)(t - t0) * F * a.npix, a.npix, p);
                if (t + 1 == t1) break;
                const Input in = load_input(a, t, p);
                const uint64_t rr = a.rec[(int64_t)t * a.npix + p];
                float mud[K][1];
#pragma unroll
                for (int k = 0; k < K; ++k) mud[k][0] = s.mud[k];
                replay_mix<K, 3>(s.muc, s.vc, in.Xc, (uint32_t)rr, alpha, a.c.v_init_c, a.c.v_min_c);
                replay_mix<K, 1>(mud, s.vd, in.Xd, (uint32_t)(rr >> 32), alpha, a.c.v_init_d, a.c.v_min_d);
#pragma unroll
                for (int k = 0; k < K; ++k) s.mud[k] = mud[k][0];
            }
            for (int t = t1 - 1; t >= t0; --t) {
                load_mv<K>(s, a.scratch + (int64_t)(t - t0) * F * a.npix, a.npix, p);
                const Input in = load_input(a, t, p);
                const int64_t o = (int64_t)t * a.npix + p;
                const uint64_t rr = a.rec[o];
                const uint32_t rc = (uint32_t)rr, rd = (uint32_t)(rr >> 32);
                float mud[K][1];
#pragma unroll
                for (int k = 0; k < K; ++k) mud[k][0] = s.mud[k];
                // the step t: post-state adjoint -> pre-state adjoint
                g_alpha += reverse_mix<K, 3>(s.muc, s.vc, in.Xc, rc, alpha, amc, avc);
                g_alpha += reverse_mix<K, 1>(mud, s.vd, in.Xd, rd, alpha, amd, avd);
                // the score Z_t on the pre-state
                const float g = a.dZ[o];
                if (rc & 1u) {
                    score_adjoint<K, 3>(s.muc, s.vc, in.Xc, rc, g, amc, avc);
                    g_lam += (double)(g * (-2.0f * lam));
                }
                if (rd & 1u) {
                    const float dd = score_adjoint<K, 1>(mud, s.vd, in.Xd, rd, g * wd, amd, avd);
                    g_lam += (double)(g * (-2.0f * lam) * wd);
                    g_wd += (double)(g * (dd - lam2));
                }
            }
        }
    }
    const double ra = block_sum(g_alpha, sh);
    const double rl = block_sum(g_lam, sh);
    const double rw = block_sum(g_wd, sh);
    if (threadIdx.x == 0) {
        a.partial[3 * blockIdx.x + 0] = ra;
        a.partial[3 * blockIdx.x + 1] = rl;
        a.partial[3 * blockIdx.x + 2] = rw;
    }
}

__global__ __launch_bounds__(kBlock) void gmm_window_reduce_kernel(const double* partial, int nblocks,
                                                                  double* out) {
    __shared__ double sh[kBlock];
    for (int i = 0; i < 3; ++i) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) acc += partial[3 * b + i];
        const double r = block_sum(acc, sh);
        if (threadIdx.x == 0) out[i] = r;
    }
}

}  // namespace

int gmm_window_blocks(int npix) { return (npix + kBlock - 1) / kBlock; }

bool gmm_window_supported(int K) { return K >= 1 && K <= 5; }

hipError_t gmm_window_launch_forward(const GmmWindowArgs& a, int K, hipStream_t s) {
    const dim3 grid(gmm_window_blocks(a.npix));
    switch (K) {
        case 1: hipLaunchKernelGGL(gmm_window_forward_kernel<1>, grid, dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL(gmm_window_forward_kernel<2>, grid, dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL(gmm_window_forward_kernel<3>, grid, dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL(gmm_window_forward_kernel<4>, grid, dim3(kBlock), 0, s, a); break;
        case 5: hipLaunchKernelGGL(gmm_window_forward_kernel<5>, grid, dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t gmm_window_launch_backward(const GmmWindowArgs& a, int K, hipStream_t s) {
    const int nb = gmm_window_blocks(a.npix);
    const dim3 grid(nb);
    switch (K) {
        case 1: hipLaunchKernelGGL(gmm_window_backward_kernel<1>, grid, dim3(kBlock), 0, s, a); break;
        case 2: hipLaunchKernelGGL(gmm_window_backward_kernel<2>, grid, dim3(kBlock), 0, s, a); break;
        case 3: hipLaunchKernelGGL(gmm_window_backward_kernel<3>, grid, dim3(kBlock), 0, s, a); break;
        case 4: hipLaunchKernelGGL(gmm_window_backward_kernel<4>, grid, dim3(kBlock), 0, s, a); break;
        case 5: hipLaunchKernelGGL(gmm_window_backward_kernel<5>, grid, dim3(kBlock), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gmm_window_reduce_kernel, dim3(1), dim3(kBlock), 0, s, a.partial, nb, a.dtheta);
    return hipGetLastError();
}

}  // namespace fgs
