// Per-tile device code of the RGB-D PBAS step (Sec. 3.2), shared by the per-frame
// kernels and the multi-stream serving kernel.
//
// Neighbour updates without races or atomics.  At frame t a background pixel x
// may write its 8-neighbour y's own value I(y,t) into a random sample of y.  All
// such writes into y carry the same value and only y itself touches its D
// history, so their order does not matter; what matters is that y's
// classification at frame t still sees the model of frame t-1.  Each pixel
// therefore records its intent (fire, direction, slot per channel, 64 bits) at
// frame t, and at frame t+1 every pixel first gathers the intents of its eight
// neighbours from a 64x4 tile plus 1-pixel halo staged in LDS and applies the
// writes aimed at it, using its stored previous value, before it classifies.
//
// Tile shape: a 256-lane workgroup covers 64 columns x 4 rows, one wavefront per
// row, one pixel per lane, so each sample-plane access of a wavefront is 256
// contiguous bytes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "fgs_internal.h"

namespace fgs {
namespace pbas {


constexpr int kTileW = 64;
constexpr int kTileH = 4;
constexpr int kBlock = kTileW * kTileH;
constexpr int kHaloW = kTileW + 2;
constexpr int kHaloH = kTileH + 2;

// 8-neighbourhood indexed by the 3-bit direction field: (dx, dy) =
// (-1,-1) (0,-1) (1,-1) (-1,0) (1,0) (-1,1) (0,1) (1,1).  The table is point
// symmetric: the opposite of direction d is 7 - d.
__device__ __forceinline__ int nb_dx(int d) { return (d == 0 || d == 3 || d == 5) ? -1 : ((d == 1 || d == 6) ? 0 : 1); }
__device__ __forceinline__ int nb_dy(int d) { return d < 3 ? -1 : (d < 5 ? 0 : 1); }

__device__ __forceinline__ uint8_t* byte_at(uint32_t* plane0, int64_t npix, int slot, int p, int j) {
    return reinterpret_cast<uint8_t*>(plane0 + (int64_t)slot * npix + p) + j;
}

// Sample planes are touched once per frame: non-temporal when the device's
// resident model state exceeds the last-level cache (see gmm_kernels.hip).
template <bool NT>
__device__ __forceinline__ uint32_t ld_sample(const uint32_t* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT>
__device__ __forceinline__ void st_sample(uint32_t* p, uint32_t v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Stage the intents of the tile and its 1-pixel halo into LDS.
__device__ __forceinline__ void stage_intents(uint64_t* lds, const uint64_t* __restrict__ intents,
                                              int x0, int y0, int H, int W) {
    for (int i = threadIdx.x; i < kHaloW * kHaloH; i += kBlock) {
        const int gx = x0 + (i % kHaloW) - 1;
        const int gy = y0 + (i / kHaloW) - 1;
        uint64_t v = 0;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) v = intents[(int64_t)gy * W + gx];
        lds[i] = v;
    }
}

// Apply the neighbour writes aimed at pixel (lx,ly) of the tile: byte stores of
// the pixel's previous value into the chosen sample slots.
__device__ __forceinline__ void apply_pending(const uint64_t* lds, int lx, int ly, uint32_t lastw,
                                              uint32_t* samples, int64_t npix, int p, int N) {
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        // the source x sits at offset delta[d] from this pixel and must have fired
        // in the opposite direction 7 - d to reach it
        const int ox = nb_dx(d), oy = nb_dy(d);
        const uint64_t v = lds[(ly + 1 + oy) * kHaloW + (lx + 1 + ox)];
        if (v == 0) continue;
        const uint32_t want = 0x8u | (uint32_t)(7 - d);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t f = (uint32_t)(v >> (16 * j)) & 0xFFFFu;
            if ((f >> 12) != want) continue;
            const uint32_t val = (lastw >> (8 * j)) & 0xFFu;
            const int slot = (int)(f & 0x3Fu);
            if ((j == 3 && val == 0u) || slot >= N) continue;  // y had no depth at that frame
            *byte_at(samples, npix, slot, p, j) = (uint8_t)val;
        }
    }
}

// One updating frame.  The pixel's N sample words live in registers between one
// dense coalesced read and one dense coalesced write of the sample planes (the
// random slot replacements are applied in registers), so no sample plane sees a
// partial-line write.  The Philox draws and the 1/T tests do not depend on the
// classification, so the candidate self-update slots are known first and their
// D-history bytes are fetched before the samples, off the critical path.
// Gather the neighbour writes aimed at pixel (lx,ly) into per-channel slot
// bit-planes: plane j, word w holds slots 32w..32w+31.  Each lane touches only its
// own words of `pend` (layout [word][lane]), so no atomics and no barrier.
template <int PW>
__device__ __forceinline__ void gather_pending(const uint64_t* lds, uint32_t* pend, int lx, int ly,
                                               int tid, uint32_t lastw, int N) {
    const bool depth_ok = (lastw >> 24) != 0u;  // y had depth at that frame
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int ox = nb_dx(d), oy = nb_dy(d);
        const uint64_t v = lds[(ly + 1 + oy) * kHaloW + (lx + 1 + ox)];
        if (v == 0) continue;
        const uint32_t want = 0x8u | (uint32_t)(7 - d);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t f = (uint32_t)(v >> (16 * j)) & 0xFFFFu;
            const int slot = (int)(f & 0x3Fu);
            if ((f >> 12) != want || slot >= N || (j == 3 && !depth_ok)) continue;
            pend[(j * PW + (slot >> 5)) * kBlock + tid] |= 1u << (slot & 31);
        }
    }
}

// LDS a tile needs: the intents halo and the pending bit-planes.
template <int NMAX>
struct PbasLds {
    static constexpr int PW = (NMAX + 31) / 32;  // words per channel bit-plane
    uint64_t halo[kHaloW * kHaloH];
    uint32_t pend[4 * PW * kBlock];
};

// One updating frame on the 64x4 tile (bx, by); all 256 lanes of the block call it.
template <int NMAX, bool NT>
__device__ __forceinline__ void pbas_tile(const PbasStepArgs& a, int bx, int by, PbasLds<NMAX>& sh) {
    constexpr int PW = PbasLds<NMAX>::PW;
    uint64_t* lds = sh.halo;
    uint32_t* pend = sh.pend;
    const int lx = threadIdx.x % kTileW, ly = threadIdx.x / kTileW;
    const int x0 = bx * kTileW, y0 = by * kTileH;
    const int x = x0 + lx, y = y0 + ly;
    const int W = a.W, H = a.H;
    const int64_t npix = a.npix;
    const int N = a.c.N;

    const int tid = threadIdx.x;
    if (a.apply_pending) {
#pragma unroll
        for (int w = 0; w < 4 * PW; ++w) pend[w * kBlock + tid] = 0u;
        stage_intents(lds, a.m.intents[(a.t - 1u) & 1u], x0, y0, H, W);
        __syncthreads();
    }
    if (x >= W || y >= H) return;
    const int p = y * W + x;

    // Ingest.
    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = load_depth(a.depth, a.depth_stride, x, y, a.W, a.H, a.depth_w, a.depth_h);
    const bool valid = dmm > 0u;
    int I[4];
    I[0] = px[0];
    I[1] = px[1];
    I[2] = px[2];
    I[3] = (int)depth_code(dmm, a.c.depth_max_mm);
    const uint32_t Iw = (uint32_t)I[0] | ((uint32_t)I[1] << 8) | ((uint32_t)I[2] << 16) | ((uint32_t)I[3] << 24);

    const float4 Rv = a.m.R[p];
    const float4 Tv = a.m.T[p];
    const uint2 Sv = a.m.S[p];
    const uint32_t lastw = a.m.last[p];
    float R[4] = {Rv.x, Rv.y, Rv.z, Rv.w};
    float T[4] = {Tv.x, Tv.y, Tv.z, Tv.w};
    int S[4] = {(int)(Sv.x & 0xFFFFu), (int)(Sv.x >> 16), (int)(Sv.y & 0xFFFFu), (int)(Sv.y >> 16)};
    const bool active[4] = {true, true, true, valid};

    // Two Philox blocks: 0 drives the self-update, 1 the neighbour update.
    const U32x4 w0 = philox4x32_10((uint32_t)p, a.t, 0u, 0u, a.c.key0, a.c.key1);
    const U32x4 w1 = philox4x32_10((uint32_t)p, a.t, 1u, 0u, a.c.key0, a.c.key1);
    const float inv16 = 1.0f / 65536.0f;

    // Self-update candidates: the 1/T test with T from before this frame.
    bool cand[4];
    int ks[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t a0 = w0.v[j];
        cand[j] = active[j] && (float)(a0 >> 16) * inv16 * T[j] < 1.0f;
        ks[j] = (int)(((a0 & 0xFFFFu) * (uint32_t)N) >> 16);
    }
    int dold[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) dold[j] = cand[j] ? (int)*byte_at(a.m.dhist, npix, ks[j], p, j) : 0;

    uint32_t sm[NMAX];
    const uint32_t* sp = a.m.samples + p;
#pragma unroll
    for (int k = 0; k < NMAX; ++k) sm[k] = k < N ? ld_sample<NT>(sp + (int64_t)k * npix) : 0u;

    // Frame t-1's neighbour writes into this pixel, before it is classified: slot k
    // of channel j takes this pixel's previous value where bit k of plane j is set.
    if (a.apply_pending) {
        gather_pending<PW>(lds, pend, lx, ly, tid, lastw, N);
        uint32_t pw[4][PW];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int w = 0; w < PW; ++w) pw[j][w] = pend[(j * PW + w) * kBlock + tid];
#pragma unroll
        for (int k = 0; k < NMAX; ++k) {
            const int w = k >> 5, b = k & 31;
            // all-ones where the bit is set, then one byte lane per channel
            const uint32_t m0 = (uint32_t)((int32_t)(pw[0][w] << (31 - b)) >> 31);
            const uint32_t m1 = (uint32_t)((int32_t)(pw[1][w] << (31 - b)) >> 31);
            const uint32_t m2 = (uint32_t)((int32_t)(pw[2][w] << (31 - b)) >> 31);
            const uint32_t m3 = (uint32_t)((int32_t)(pw[3][w] << (31 - b)) >> 31);
            const uint32_t bm = (m0 & 0x000000FFu) | (m1 & 0x0000FF00u) | (m2 & 0x00FF0000u) | (m3 & 0xFF000000u);
            sm[k] = (sm[k] & ~bm) | (lastw & bm);
        }
    }

    // Classification: an integer distance d is within R iff d <= ceil(R) - 1.
    int thr[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) thr[j] = (int)fminf(ceilf(R[j]), 256.0f) - 1;
    int cnt[4] = {0, 0, 0, 0};
    int dmn[4] = {255, 255, 255, 255};
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        if (k < N) {
            const uint32_t s = sm[k];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int dd = abs((int)((s >> (8 * j)) & 0xFFu) - I[j]);
                cnt[j] += dd <= thr[j] ? 1 : 0;
                dmn[j] = min(dmn[j], dd);
            }
            const int b3 = (int)(s >> 24);
            const int dd = b3 != 0 ? abs(b3 - I[3]) : 256;  // empty depth slot: never within R
            cnt[3] += dd <= thr[3] ? 1 : 0;
            dmn[3] = min(dmn[3], dd);
        }
    }
    bool F[4], upd[4];
    bool fg = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        F[j] = active[j] && cnt[j] < a.c.min_matches;
        fg = fg || F[j];
        upd[j] = cand[j] && !F[j];
    }
    a.m.mask[p] = fg ? (uint8_t)255 : (uint8_t)0;

    // Self-update: sample slot ks[j] takes I_j, its D slot takes d_min.
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        uint32_t v = sm[k];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (upd[j] && ks[j] == k) v = (v & ~(0xFFu << (8 * j))) | ((uint32_t)I[j] << (8 * j));
        sm[k] = v;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (upd[j]) {
            S[j] = S[j] - dold[j] + dmn[j];
            *byte_at(a.m.dhist, npix, ks[j], p, j) = (uint8_t)dmn[j];
        }

    // Neighbour update with probability 1/T (T from before this frame): record the intent.
    uint64_t intent = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!active[j] || F[j]) continue;
        const uint32_t a1 = w1.v[j];
        if ((float)(a1 >> 16) * inv16 * T[j] < 1.0f) {
            const int d = (int)((a1 >> 13) & 7u);
            const int nx = x + nb_dx(d), ny = y + nb_dy(d);
            if (nx >= 0 && nx < W && ny >= 0 && ny < H) {
                const uint32_t slot = ((a1 & 0x1FFFu) * (uint32_t)N) >> 13;
                intent |= (uint64_t)(0x8000u | ((uint32_t)d << 12) | slot) << (16 * j);
            }
        }
    }

    // Decision threshold and update rate.
    const float rdn = 1.0f - a.c.R_incdec, rup = 1.0f + a.c.R_incdec;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!active[j]) continue;
        const float dbar = (float)S[j] / (float)N;
        const float r = (R[j] > dbar * a.c.R_scale) ? R[j] * rdn : R[j] * rup;
        R[j] = fmaxf(r, a.c.R_lower[j]);
        const float tt = F[j] ? T[j] + a.c.T_inc / dbar : T[j] - a.c.T_dec / dbar;
        T[j] = fminf(fmaxf(tt, a.c.T_lower), a.c.T_upper);
    }

    uint32_t* so = a.m.samples + p;
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
        if (k < N) st_sample<NT>(so + (int64_t)k * npix, sm[k]);
    a.m.R[p] = make_float4(R[0], R[1], R[2], R[3]);
    a.m.T[p] = make_float4(T[0], T[1], T[2], T[3]);
    a.m.S[p] = make_uint2((uint32_t)S[0] | ((uint32_t)S[1] << 16), (uint32_t)S[2] | ((uint32_t)S[3] << 16));
    a.m.last[p] = Iw;
    a.m.intents[a.t & 1u][p] = intent;
}

// Frames 0..N-1: sample slot t takes the frame; the mask is empty.
__device__ __forceinline__ void fill_pixel(const PbasStepArgs& a, int p) {
    const int y = p / a.W, x = p - (p / a.W) * a.W;
    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = load_depth(a.depth, a.depth_stride, x, y, a.W, a.H, a.depth_w, a.depth_h);
    const uint32_t Iw = (uint32_t)px[0] | ((uint32_t)px[1] << 8) | ((uint32_t)px[2] << 16) |
                        (depth_code(dmm, a.c.depth_max_mm) << 24);
    a.m.samples[(int64_t)a.t * a.npix + p] = Iw;
    a.m.last[p] = Iw;
    a.m.mask[p] = 0;
}

}  // namespace pbas
}  // namespace fgs
