// Per-tile device code of the RGB-D PBAS step (Sec. 3.2), shared by the per-frame
// kernels and the multi-stream serving kernel.
//
// Neighbour updates without races or atomics on HBM.  At frame t a background
// pixel x may write its 8-neighbour y's own value I(y,t) into a random sample of
// y.  All such writes into y carry the same value and only y itself touches its D
// history, so their order does not matter; what matters is that y's
// classification at frame t still sees the model of frame t-1.  Each pixel
// therefore records at frame t which channels fired (one byte), and at frame t+1
// each tile recomputes the direction and slot of every write aimed into it from
// the sources' Philox draws, collects them in LDS, and every pixel applies them,
// using its stored previous value, before it classifies.
//
// Tile shape: a 256-lane workgroup covers 64 columns x 4 rows, one wavefront per
// row, one pixel per lane, so each sample access of a wavefront (a 16-byte quad
// of slots per lane) is 1 KiB of contiguous memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "fgs_internal.h"

namespace fgs {
namespace pbas {

constexpr int kTileW = kPbasTileW;
constexpr int kTileH = kPbasTileH;
constexpr int kBlock = kTileW * kTileH;
constexpr int kHaloW = kTileW + 2;
constexpr int kHaloH = kTileH + 2;

// 8-neighbourhood indexed by the 3-bit direction field: (dx, dy) =
// (-1,-1) (0,-1) (1,-1) (-1,0) (1,0) (-1,1) (0,1) (1,1).  The table is point
// symmetric: the opposite of direction d is 7 - d.  dx + 1 and dy + 1 are packed two
// bits per direction (bits 2d, 2d + 1), so a lookup is a bit-field extract with no
// branch: dx + 1 = 0,1,2,0,2,0,1,2 -> 0x9224; dy + 1 = 0,0,0,1,1,2,2,2 -> 0xA940.
__device__ __forceinline__ int nb_dx(int d) { return (int)((0x9224u >> (2 * d)) & 3u) - 1; }
__device__ __forceinline__ int nb_dy(int d) { return (int)((0xA940u >> (2 * d)) & 3u) - 1; }

// D history: slot k of pixel p is the 32-bit word k * npix + p (one byte per channel).
__device__ __forceinline__ uint8_t* byte_at(uint32_t* plane0, int64_t npix, int slot, int p, int j) {
    return reinterpret_cast<uint8_t*>(plane0 + (int64_t)slot * npix + p) + j;
}

// Sample storage: slot k of pixel p is word k & 3 of the 16-byte element
// (k >> 2) * npix + p of the sample array ("quad planes" of four slots), so a
// wavefront moves 1 KiB contiguous per load or store instruction.  Slots from N
// up to the next multiple of 4 are padding and stay zero.
__device__ __forceinline__ uint8_t* sample_byte(uint32_t* samples, int64_t npix, int slot, int p, int j) {
    return reinterpret_cast<uint8_t*>(samples + (((int64_t)(slot >> 2) * npix + p) << 2) + (slot & 3)) + j;
}

// Sample quads are touched once per frame: non-temporal when the device's
// resident model state exceeds the last-level cache (see gmm_kernels.hip).  A quad
// plane is read and written through a raw buffer resource whose base is the
// tile's first pixel in that plane (uniform across the wavefront) with the
// lane's 32-bit byte offset from there, so no per-quad address is held in vector
// registers; the range ends at the plane's end, and the hardware drops any
// access beyond it.
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit buffer, gfx9 family

typedef uint32_t u32x4 __attribute__((__vector_size__(4 * sizeof(uint32_t))));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t quad_rsrc(const uint32_t* tile0, int64_t npix, uint32_t range,
                                                           int q) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(tile0) + (size_t)q * (size_t)npix * 4u,
                                             (short)0, (int)range, kBufferWord3);
}
template <bool NT>
__device__ __forceinline__ u32x4 ld_quad(const uint32_t* tile0, int64_t npix, uint32_t range, int q, uint32_t voff) {
    return __builtin_amdgcn_raw_buffer_load_b128(quad_rsrc(tile0, npix, range, q), voff, 0, NT ? 2 : 0);
}
template <bool NT>
__device__ __forceinline__ void st_quad(uint32_t* tile0, int64_t npix, uint32_t range, int q, uint32_t voff,
                                        u32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(v, quad_rsrc(tile0, npix, range, q), voff, 0, NT ? 2 : 0);
}

// Where channel j of pixel q sends its neighbour write at frame t: direction and
// slot from the Philox block 1 word j of (q, t), as the pixel drew them then.
__device__ __forceinline__ void intent_of(uint32_t word, int N, int& dir, int& slot) {
    dir = (int)((word >> 13) & 7u);
    slot = (int)(__umul24(word & 0x1FFFu, (uint32_t)N) >> 13);  // < N; 13 x 7 bits: 24-bit multiply
}

// Pending writes into a tile pixel are kept as slot bit-words: for sample slot k
// of channel j, bit 8*j + (k & 7) of word k >> 3.  Shifting word k >> 3 right by
// k & 7 and masking with 0x01010101 leaves one bit per channel in the low bit of
// that channel's byte, which a 16-bit lane multiply by 0xFF widens into a byte
// mask of the sample word (slot_byte_mask, for run-time slot indices); the unrolled
// slot loops merge with a byte permute instead (merge_slot, one instruction fewer).
constexpr uint32_t kLowBits = 0x01010101u;

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 h2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t w32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// Whether two float4 differ in any bit.
__device__ __forceinline__ bool differs(float4 a, float4 b) {
    return (__float_as_uint(a.x) ^ __float_as_uint(b.x)) | (__float_as_uint(a.y) ^ __float_as_uint(b.y)) |
           (__float_as_uint(a.z) ^ __float_as_uint(b.z)) | (__float_as_uint(a.w) ^ __float_as_uint(b.w));
}

// Byte mask of the channels whose bit is set for slot k in bit-word `word`.
__device__ __forceinline__ uint32_t slot_byte_mask(uint32_t word, int k) {
    const uint32_t bits = (word >> (k & 7)) & kLowBits;
    return w32(h2(bits) * (u16x2){0xFF, 0xFF});
}

// Slot k's sample word with the bytes of `val` in place of those whose channel bit is
// set for slot k in bit-word `word`, the rest from `cur`: the bits are shifted to bit 2
// of their channel's byte, which then selects byte j + 4 (val) instead of byte j (cur)
// in a byte permute.  (k is a constant in the unrolled slot loops, so the shift is one
// instruction in a fixed direction.)  `byte_ids` holds 0x03020100.
__device__ __forceinline__ uint32_t merge_slot(uint32_t cur, uint32_t val, uint32_t word, int k,
                                               uint32_t byte_ids) {
    const int s = k & 7;
    const uint32_t x = s >= 2 ? word >> (s - 2) : word << (2 - s);
    uint32_t sel;  // (x & 0x04040404) | byte_ids in one three-input logic instruction
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0xea" : "=v"(sel) : "v"(x), "s"(0x04040404u), "v"(byte_ids));
    return __builtin_amdgcn_perm(val, cur, sel);
}

// LDS a tile needs: the pending bit-words, word w of tile pixel i at [w][i].
template <int NMAX>
struct PbasLds {
    static constexpr int NW = (NMAX + 7) / 8;  // bit-words per pixel
    uint32_t pend[NW * kBlock];
};

// Frame t-1's neighbour writes aimed at this tile, scattered from their sources:
// every pixel of the tile and of its 1-pixel halo is read once (its fire byte); a
// source that fired recomputes its Philox block 1 of frame t-1 for the direction
// and slot, and each write that lands inside the tile sets its (slot, channel) bit
// in the destination's bit-words with an LDS atomic OR.  Whether the destination
// had depth at t-1 is checked by the destination.
//
// Lane tid reads halo pixels tid and tid + kBlock (row-major over the
// (kTileW + 2) x (kTileH + 2) halo); the bytes are loaded first and scattered
// later, so the loads overlap the tile's other reads.
static_assert(kHaloW * kHaloH <= 2 * kBlock, "two halo pixels per lane");

struct FireIn {
    uint32_t fb[2];  // fire byte (0: nothing to scatter, or no such pixel)
    int q[2];        // its pixel index
};

__device__ __forceinline__ FireIn load_fire(const uint8_t* fire, int x0, int y0, int H, int W) {
    FireIn f;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int i = (int)threadIdx.x + r * kBlock;
        const int hx = i % kHaloW, hy = i / kHaloW;
        const int gx = x0 + hx - 1, gy = y0 + hy - 1;
        f.fb[r] = 0u;
        f.q[r] = gy * W + gx;
        if (i < kHaloW * kHaloH && gx >= 0 && gx < W && gy >= 0 && gy < H) f.fb[r] = fire[f.q[r]];
    }
    return f;
}

template <int NMAX>
__device__ __forceinline__ void scatter_fired(PbasLds<NMAX>& sh, const FireIn& f, int N, uint32_t t_prev,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const uint32_t fb = f.fb[r] & 0xFu;  // the high nibble carries R flags (pbas_tile)
        if (fb == 0u) continue;
        const int i = (int)threadIdx.x + r * kBlock;
        const int hx = i % kHaloW, hy = i / kHaloW;
        const U32x4 w1 = philox4x32_10((uint32_t)f.q[r], t_prev, 1u, 0u, k0, k1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!((fb >> j) & 1u)) continue;
            int d, slot;
            intent_of(w1.v[j], N, d, slot);
            const int tx = hx - 1 + nb_dx(d), ty = hy - 1 + nb_dy(d);
            if ((unsigned)tx >= (unsigned)kTileW || (unsigned)ty >= (unsigned)kTileH) continue;
            __hip_atomic_fetch_or(&sh.pend[(slot >> 3) * kBlock + ty * kTileW + tx],
                                  1u << (8 * j + (slot & 7)), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// One updating frame on the 64x4 tile (bx, by); all 256 lanes of the block call it.
// N lies in [NLO, NMAX]: slots below NLO need no run-time bound check.
//
// The pixel's N sample words live in registers between one dense coalesced read
// and the write-back of the sample quad planes: frame t-1's neighbour writes and
// this frame's self-update are merged in registers slot by slot (byte permutes), and
// a quad goes back to memory, in whole 64-byte sectors, only where a byte of it
// changed in one of the sector's 4 pixels, so no quad plane sees a partial-sector
// write.  Every read of the frame
// is issued before the scatter of the neighbour writes (fire bytes first, then
// the pixel's state and samples), and since the Philox draws and the 1/T tests
// do not depend on the classification, the candidate self-update slots are known
// early and their D-history bytes are fetched during the scatter, off the critical
// path.
//
// Classification runs two channels per 32-bit word (16-bit lanes: R|B and G|D).
// The depth lane holds code - 1, so an empty depth slot (code 0) becomes 0xFFFF,
// whose distance to any valid code is above every threshold and every d_min.
template <int NMAX, int NLO, bool NT>
__device__ __forceinline__ void pbas_tile(const PbasStepArgs& a, int bx, int by, PbasLds<NMAX>& sh) {
    static_assert(NLO >= 1 && NLO <= NMAX, "bad register capacity class");
    constexpr int NW = PbasLds<NMAX>::NW;
    const int tid = threadIdx.x;
    const int lx = tid % kTileW, ly = tid / kTileW;
    const int x0 = bx * kTileW, y0 = by * kTileH;
    const int W = a.W, H = a.H;
    const int64_t npix = a.npix;
    const int N = a.c.N;
    // Every lane issues its reads before the scatter so that their latency overlaps
    // it; a lane past the image edge reads the tile origin's pixel (always inside)
    // and leaves after the scatter without writing anything.
    const bool inside = x0 + lx < W && y0 + ly < H;
    const int x = inside ? x0 + lx : x0, y = inside ? y0 + ly : y0;
    const int p = y * W + x;

    FireIn fin = {{0u, 0u}, {0, 0}};
    if (a.apply_pending) {
#pragma unroll
        for (int w = 0; w < NW; ++w) sh.pend[w * kBlock + tid] = 0u;
        fin = load_fire(a.m.fire[(a.t - 1u) & 1u], x0, y0, H, W);
    }

    // The pixel's own reads: T first (the self-update draws need it), then R, S, the
    // previous value and the frame.  The scheduling fences keep them ahead of the
    // sample reads: loads complete in order, so the D-history reads that wait for T
    // then need not wait for the samples.
    // The previous value sits in padding slot N when the model put it there (N >= 33,
    // not a multiple of 4) and the class can select it from registers (at most 7
    // candidate slots).  Smaller classes keep it in its plane: there the select would
    // cost occupancy.
    constexpr bool kPadOK = NMAX - NLO <= 7 && NMAX >= 36;
    const bool in_pad = kPadOK && a.m.last_in_pad;
    // Frame t-1 left in the high nibble of the pixel's fire byte which channels' R equal
    // their lower bound exactly (where R sits on a static background); where all four do,
    // R is known without reading it.  Read first, so that the R read, issued after the
    // samples, need not wait for anything later.
    const uint32_t rflags = a.apply_pending ? (uint32_t)a.m.fire[(a.t - 1u) & 1u][p] >> 4 : 0u;
    const float4 Tv = a.m.T[p];
    const uint2 Sv = a.m.S[p];
    uint32_t lastw = in_pad ? 0u : a.m.last[p];
    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = load_depth(a.depth, a.depth_stride, x, y, a.W, a.H, a.depth_w, a.depth_h);
    const uint32_t I0 = px[0], I1 = px[1], I2 = px[2];
    __builtin_amdgcn_sched_barrier(0);

    // Quads 4q < N hold samples (the first NLO slots need no run-time test);
    // padding slots come in as zero and are never used.
    uint32_t sm[NMAX];
    const int64_t p0 = (int64_t)y0 * W + x0;                     // tile origin, < npix
    const uint32_t* stile = a.m.samples + p0 * 4;
    const int64_t qleft = (npix - p0) * 16;                       // bytes from the origin to the plane end
    const uint32_t qrange = qleft > 0xFFFFFFFFll ? 0xFFFFFFFFu : (uint32_t)qleft;
    const uint32_t voff = (uint32_t)(p - p0) * 16u;               // p - p0 < npix <= 2^28
#pragma unroll
    for (int q = 0; q < NMAX / 4; ++q) {
        if (4 * q < NLO || 4 * q < N) {
            const u32x4 v = ld_quad<NT>(stile, npix, qrange, q, voff);
#pragma unroll
            for (int i = 0; i < 4; ++i) sm[4 * q + i] = v[i];
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) sm[4 * q + i] = 0u;
        }
    }
    const float4 Rv = rflags == 0xFu ? make_float4(a.c.R_lower[0], a.c.R_lower[1], a.c.R_lower[2], a.c.R_lower[3])
                                     : a.m.R[p];

    __builtin_amdgcn_sched_barrier(0);

    // Ingest (the depth code needs the depth read; computed once every read is issued).
    const bool valid = dmm > 0u;
    const uint32_t I3 = depth_code(dmm, a.c.depth_max_mm);
    const uint32_t Iw = I0 | (I1 << 8) | (I2 << 16) | (I3 << 24);
    float R[4] = {Rv.x, Rv.y, Rv.z, Rv.w};
    float T[4] = {Tv.x, Tv.y, Tv.z, Tv.w};
    int S[4] = {(int)(Sv.x & 0xFFFFu), (int)(Sv.x >> 16), (int)(Sv.y & 0xFFFFu), (int)(Sv.y >> 16)};
    const bool active[4] = {true, true, true, valid};

    // Block 0 of the Philox draws drives the self-update.
    const U32x4 w0 = philox4x32_10((uint32_t)p, a.t, 0u, 0u, a.c.key0, a.c.key1);
    const float inv16 = 1.0f / 65536.0f;

    if (a.apply_pending) {
        __syncthreads();  // bit-words cleared
        scatter_fired<NMAX>(sh, fin, N, a.t - 1u, a.c.key0, a.c.key1);
    }

    // Self-update candidates: the 1/T test with T from before this frame.
    bool cand[4];
    int ks[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t a0 = w0.v[j];
        cand[j] = active[j] && (float)(a0 >> 16) * inv16 * T[j] < 1.0f;
        ks[j] = (int)(__umul24(a0 & 0xFFFFu, (uint32_t)N) >> 16);  // 16 x 7 bits: 24-bit multiply
    }
    int dold[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) dold[j] = cand[j] ? (int)*byte_at(a.m.dhist, npix, ks[j], p, j) : 0;

    if (a.apply_pending) __syncthreads();  // every write aimed at the tile recorded
    if (!inside) return;

    if (in_pad) {
#pragma unroll
        for (int k = NLO; k < NMAX; ++k)
            if (k == N) lastw = sm[k];
    }

    // Classification: an integer distance d is within R iff d < min(ceil(R), 256)
    // (no d is within a threshold R <= 0 or NaN).
    uint32_t lim[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) lim[j] = R[j] > 0.0f ? (uint32_t)fminf(ceilf(R[j]), 256.0f) : 0u;
    const u16x2 I_rb = h2(I0 | (I2 << 16));
    const u16x2 I_gd = h2(I1 | (((I3 - 1u) & 0xFFFFu) << 16));
    const u16x2 L_rb = h2(lim[0] | (lim[2] << 16));
    const u16x2 L_gd = h2(lim[1] | (lim[3] << 16));
    const u16x2 cap = {0x200, 0x200};
    const u16x2 one5 = {15, 15};
    const u16x2 dep1 = {0, 1};
    u16x2 cnt_rb = {0, 0}, cnt_gd = {0, 0};
    u16x2 dmn_rb = {255, 255}, dmn_gd = {255, 255};

    // Frame t-1's neighbour writes into this pixel come first: slot k of channel j
    // takes this pixel's previous value where its bit is set.
    uint32_t pw[NW];
    const uint32_t keep = (lastw >> 24) != 0u ? 0xFFFFFFFFu : 0x00FFFFFFu;  // depth at t-1?
#pragma unroll
    for (int w = 0; w < NW; ++w) pw[w] = a.apply_pending ? sh.pend[w * kBlock + tid] & keep : 0u;
    // Bit q of `dirty`: some byte of sample quad q changed, by the neighbour writes
    // merged here (each merged slot compared with the word it replaces, four slots to a
    // quad; the empty asm keeps each quad's test next to its slots, where the words are
    // in registers anyway), then by the previous value and the self-update below.
    uint32_t dirty = 0u, chg = 0u;
    uint32_t byte_ids;  // an opaque register, so the constant is not rematerialised per merge
    asm("v_mov_b32 %0, 0x03020100" : "=v"(byte_ids));
#pragma unroll
    for (int k = 0; k < NMAX; ++k) {
        // Keep the per-slot work next to its sample: without the fence the scheduler
        // runs the mask arithmetic of every slot ahead of the loads and holds N more
        // registers.
        if ((k & 7) == 0) __builtin_amdgcn_sched_barrier(0);
        const uint32_t before = sm[k];
        sm[k] = merge_slot(before, lastw, pw[k >> 3], k, byte_ids);
        chg |= sm[k] ^ before;
        if ((k & 3) == 3) {
            dirty |= (chg != 0u ? 1u : 0u) << (k >> 2);
            chg = 0u;
            asm volatile("" : "+v"(dirty));
        }
        if (k < NLO || k < N) {
            const uint32_t s = sm[k];
            // byte permutes: R|B and G|D in 16-bit lanes (depth code - 1, empty -> 0xFFFF)
            const u16x2 s_rb = h2(__builtin_amdgcn_perm(0u, s, 0x0C020C00u));
            const u16x2 s_gd = h2(__builtin_amdgcn_perm(0u, s, 0x0C030C01u)) - dep1;
            const u16x2 d_rb = __builtin_elementwise_max(s_rb, I_rb) - __builtin_elementwise_min(s_rb, I_rb);
            const u16x2 d_gd = __builtin_elementwise_max(s_gd, I_gd) - __builtin_elementwise_min(s_gd, I_gd);
            dmn_rb = __builtin_elementwise_min(dmn_rb, d_rb);
            dmn_gd = __builtin_elementwise_min(dmn_gd, d_gd);
            // (min(d, 512) - lim) is negative, bit 15 set, iff d < lim
            cnt_rb = cnt_rb + ((d_rb - L_rb) >> one5);
            cnt_gd = cnt_gd + ((__builtin_elementwise_min(d_gd, cap) - L_gd) >> one5);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    const int cnt[4] = {cnt_rb.x, cnt_gd.x, cnt_rb.y, cnt_gd.y};
    const int dmn[4] = {dmn_rb.x, dmn_gd.x, dmn_rb.y, dmn_gd.y};
    bool F[4], upd[4];
    bool fg = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        F[j] = active[j] && cnt[j] < a.c.min_matches;
        fg = fg || F[j];
        upd[j] = cand[j] && !F[j];
    }
    a.m.mask[p] = fg ? (uint8_t)255 : (uint8_t)0;

    // A D-history byte is written only when it changes: on a static background d_min is
    // mostly 0 or 1 and often equals the byte it replaces, and each write that is left
    // out saves a partial-sector write to HBM.
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (upd[j]) {
            S[j] = S[j] - dold[j] + dmn[j];
            if (dold[j] != dmn[j]) *byte_at(a.m.dhist, npix, ks[j], p, j) = (uint8_t)dmn[j];
        }

    // Neighbour update with probability 1/T (T from before this frame): record that
    // channel j fired; block 1 of the draws drives it, and the next frame's tiles
    // recompute its direction and slot from the same block.
    const U32x4 w1 = philox4x32_10((uint32_t)p, a.t, 1u, 0u, a.c.key0, a.c.key1);
    uint32_t fire = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (!active[j] || F[j]) continue;
        const uint32_t a1 = w1.v[j];
        if ((float)(a1 >> 16) * inv16 * T[j] < 1.0f) {
            const int d = (int)((a1 >> 13) & 7u);
            const int nx = x + nb_dx(d), ny = y + nb_dy(d);
            if (nx >= 0 && nx < W && ny >= 0 && ny < H) fire |= 1u << j;
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
        const float q = (F[j] ? a.c.T_inc : a.c.T_dec) / dbar;  // one division, not two and a select
        const float tt = F[j] ? T[j] + q : T[j] - q;
        T[j] = fminf(fmaxf(tt, a.c.T_lower), a.c.T_upper);
    }

    // Self-update: sample slot ks[j] takes I_j (from bit-words built in registers,
    // merged as above), quad by quad right before the quad's store, so that each quad's
    // words die at its store.  A 64-byte sector of a quad plane holds 4 consecutive
    // pixels (lanes 4i..4i+3 of a tile row): a quad's store is left out only where no
    // byte of it changed in any of the 4, so the writes that remain cover whole sectors.
    // Lanes past the image edge have left and can only add bits to the vote (a store
    // too many, never one too few).
    // (Up to 40 slots: for more, the bits' registers would cost occupancy.)
    constexpr bool kSkipClean = NMAX <= 40;
    // The self-update's bit-words are built in the lane's own LDS words (read into pw
    // before the classification, touched by no other lane since the scatter's barrier):
    // cleared, then one OR per updating channel, then read back.
    uint32_t sw[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) sh.pend[w * kBlock + tid] = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (upd[j])
            __hip_atomic_fetch_or(&sh.pend[(ks[j] >> 3) * kBlock + tid], 1u << (8 * j + (ks[j] & 7)),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int w = 0; w < NW; ++w) sw[w] = sh.pend[w * kBlock + tid];
    if (in_pad) {
#pragma unroll
        for (int k = NLO; k < NMAX; ++k)
            if (k == N) {
                dirty |= (sm[k] != Iw ? 1u : 0u) << (k >> 2);
                sm[k] = Iw;
            }
    }
    // The store loop rebuilds each quad plane's descriptor (a few scalar
    // instructions) rather than keeping them alive across the frame; the empty asm
    // hides that the base is the one the loads used.
    uint32_t* sbase = a.m.samples + p0 * 4;
    asm volatile("" : "+s"(sbase));
#pragma unroll
    for (int q = 0; q < NMAX / 4; ++q) {
        if (!(4 * q < NLO || 4 * q < N)) continue;
        uint32_t c = 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * q + i;
            const uint32_t before = sm[k];
            sm[k] = merge_slot(before, Iw, sw[k >> 3], k, byte_ids);
            c |= sm[k] ^ before;
        }
        int d = (int)(((dirty >> q) & 1u) | (c != 0u ? 1u : 0u));
        if (kSkipClean) {  // OR over each group of 4 lanes (quad permutes [1,0,3,2], [2,3,0,1])
            d |= __builtin_amdgcn_update_dpp(0, d, 0xB1, 0xF, 0xF, false);
            d |= __builtin_amdgcn_update_dpp(0, d, 0x4E, 0xF, 0xF, false);
        }
        if (!kSkipClean || d) {
            const u32x4 v = {sm[4 * q], sm[4 * q + 1], sm[4 * q + 2], sm[4 * q + 3]};
            st_quad<NT>(sbase, npix, qrange, q, voff, v);
        }
    }
    // R, T and S are written only where they changed (bit for bit): on a static
    // background R and T sit at their lower bounds and S moves only with D.
    {
        const float4 Rn = make_float4(R[0], R[1], R[2], R[3]);
        const float4 Tn = make_float4(T[0], T[1], T[2], T[3]);
        const uint2 Sn = make_uint2((uint32_t)S[0] | ((uint32_t)S[1] << 16), (uint32_t)S[2] | ((uint32_t)S[3] << 16));
        if (differs(Rn, Rv)) a.m.R[p] = Rn;
        if (differs(Tn, Tv)) a.m.T[p] = Tn;
        if (Sn.x != Sv.x || Sn.y != Sv.y) a.m.S[p] = Sn;
    }
    if (!in_pad) a.m.last[p] = Iw;
    uint32_t rfl = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) rfl |= (__float_as_uint(R[j]) == __float_as_uint(a.c.R_lower[j]) ? 1u : 0u) << j;
    a.m.fire[a.t & 1u][p] = (uint8_t)(fire | (rfl << 4));
}

// Frames 0..N-1: sample slot t takes the frame; the mask is empty.
__device__ __forceinline__ void fill_pixel(const PbasStepArgs& a, int p) {
    const int y = p / a.W, x = p - (p / a.W) * a.W;
    const uint8_t* px = a.rgb + (int64_t)y * a.rgb_stride + 3 * x;
    const uint32_t dmm = load_depth(a.depth, a.depth_stride, x, y, a.W, a.H, a.depth_w, a.depth_h);
    const uint32_t Iw = (uint32_t)px[0] | ((uint32_t)px[1] << 8) | ((uint32_t)px[2] << 16) |
                        (depth_code(dmm, a.c.depth_max_mm) << 24);
    *reinterpret_cast<uint32_t*>(sample_byte(a.m.samples, a.npix, (int)a.t, p, 0)) = Iw;
    if (a.m.last_in_pad)
        *reinterpret_cast<uint32_t*>(sample_byte(a.m.samples, a.npix, a.c.N, p, 0)) = Iw;
    else
        a.m.last[p] = Iw;
    a.m.mask[p] = 0;
}

}  // namespace pbas
}  // namespace fgs
