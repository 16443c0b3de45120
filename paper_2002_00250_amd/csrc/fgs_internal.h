// Internal declarations of libfgs: model object, kernel argument blocks and the
// host-side launch wrappers each kernel file exports to the runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fgs.h"

namespace fgs {

// ------------------------------------------------------------- batches ----
// Up to kBatchMax models of one kind and class stepped by one launch (their
// arguments travel by value): workgroup w belongs to model i when
// first[i] <= w < first[i + 1], first[0] = 0, first[n] = the grid size.  One launch
// over many independent models has one ramp-up and one drain instead of one each.
constexpr int kBatchMax = 8;

// The PBAS step's tile: a 256-lane workgroup covers kPbasTileW x kPbasTileH pixels, one
// pixel per lane (the host sizes grids and serving descriptors with the same shape).
constexpr int kPbasTileW = 64;
constexpr int kPbasTileH = 4;

// ---------------------------------------------------------------- GMM ----
// Device layout: per pixel, Kc "core" float4 planes (mu_r, mu_g, mu_b, v) of the
// colour Gaussians by rank, then E "extra" float4 planes holding, in order, the
// floats w_c[Kc], w_d[Kd], (mu_d, v_d)[Kd] and, with per-channel colour variances,
// (v_g, v_b)[Kc] (v in the core plane is then the red one), zero padded.  Plane i
// of pixel p is at state[i*npix + p]: every access is one 16-byte load or store per
// lane, a wavefront touching 1 KiB of contiguous memory.
__host__ __device__ inline int gmm_extra_planes(int Kc, int Kd, int var_mode) {
    return (Kc + 3 * Kd + (var_mode ? 2 * Kc : 0) + 3) / 4;
}
__host__ __device__ inline int gmm_planes(int Kc, int Kd, int var_mode) { return Kc + gmm_extra_planes(Kc, Kd, var_mode); }
// Float index of a field among the extra planes (float i sits in plane Kc + i/4, lane i%4).
__host__ __device__ constexpr int gmm_x_wc(int, int, int k) { return k; }
__host__ __device__ constexpr int gmm_x_wd(int Kc, int, int k) { return Kc + k; }
__host__ __device__ constexpr int gmm_x_mud(int Kc, int Kd, int k) { return Kc + Kd + 2 * k; }
__host__ __device__ constexpr int gmm_x_vd(int Kc, int Kd, int k) { return Kc + Kd + 2 * k + 1; }
__host__ __device__ constexpr int gmm_x_vg(int Kc, int Kd, int k) { return Kc + 3 * Kd + 2 * k; }
__host__ __device__ constexpr int gmm_x_vb(int Kc, int Kd, int k) { return Kc + 3 * Kd + 2 * k + 1; }
bool gmm_supported(int Kc, int Kd);

struct GmmConsts {
    float alpha, lam, T_bg, w_init, v_init_c, v_min_c, v_init_d, v_min_d, w_depth;
    uint32_t depth_max_mm;
    int32_t rho_mode;    // matched-Gaussian rate: 0 alpha, 1 alpha / w, 2 alpha * eta
    int32_t decision;    // 1: scaled Eq. (1) density product below density_threshold
    float density_scale, density_threshold;
    int32_t var_mode;    // 1: per-channel colour variances (v_init_c, v_min_c per channel)
};

struct GmmStepArgs {
    float4* state;
    int32_t streaming;  // 1: non-temporal state traffic (working set beyond the last-level cache)
    uint8_t* mask;
    const uint8_t* rgb;
    const uint8_t* depth;  // uint16 rows, addressed in bytes
    int64_t rgb_stride, depth_stride;
    int32_t H, W, npix;
    int32_t depth_h, depth_w;  // 0: depth is H x W; else its size, upscaled to H x W
    GmmConsts c;
};

// Capacity NB: a single push uses NB = 1 (small kernel arguments, one launch's
// latency as before batching), batches of 2..kBatchMax use NB = kBatchMax.
template <int NB>
struct GmmBatch {
    int32_t n;
    int32_t first[NB + 1];
    GmmStepArgs a[NB];
};

hipError_t gmm_launch_init(float4* state, int Kc, int Kd, int npix, const GmmConsts& c,
                           hipStream_t s);
hipError_t gmm_launch_step(const GmmStepArgs& a, int Kc, int Kd, hipStream_t s);
// One launch over n <= kBatchMax models with the same Kc, Kd, cache policy and
// kernel variant (gmm_batch_key equal).
hipError_t gmm_launch_step_batch(const GmmStepArgs* a, int n, int Kc, int Kd, hipStream_t s);
int gmm_batch_key(const GmmStepArgs& a, int Kc, int Kd);
// canonical planar float32 <-> device layout
hipError_t gmm_launch_export(const float4* state, float* out, int Kc, int Kd, int var_mode, int npix,
                             hipStream_t s);
hipError_t gmm_launch_import(float4* state, const float* in, int Kc, int Kd, int var_mode, int npix,
                             hipStream_t s);

// --------------------------------------------------------- GMM adjoint ----
// A window of T frames from a fresh model; checkpoints every E frames.  Frames
// are dense device arrays rgb[T][npix][3], depth[T][npix].  Snapshot planes hold
// means and variances only (6K floats per pixel).
struct GmmWindowArgs {
    int32_t T, H, W, npix, E, nseg;
    GmmConsts c;            // alpha, lam, w_depth unused: theta comes from device memory
    const float* theta;     // device [3]: alpha, lambda, w_depth
    const uint8_t* rgb;
    const uint16_t* depth;
    float* Z;               // [T][npix] pre-update scores (0 where no term)
    uint8_t* has;           // [T][npix] 1 where Z has a term
    uint64_t* rec;          // [T][npix] recorded discrete choices
    float* ckpt;            // [nseg][6K][npix]
    float* scratch;         // [E][6K][npix]
    const float* dZ;        // [T][npix]
    double* partial;        // [blocks][3]
    double* dtheta;         // [3]
};
bool gmm_window_supported(int K);
int gmm_window_blocks(int npix);
hipError_t gmm_window_launch_forward(const GmmWindowArgs& a, int K, hipStream_t s);
hipError_t gmm_window_launch_backward(const GmmWindowArgs& a, int K, hipStream_t s);

// --------------------------------------------------------------- PBAS ----
// Device layout: samples in ceil(N/4) planes of 16-byte quads (slot k of pixel p
// = word k & 3 of quad (k >> 2) * npix + p; padding slots zero), dhist[N] uint32
// planes (a sample and a D word hold bytes R,G,B,depth), R and
// T as one float4 per pixel, S as four uint16 per pixel (uint2), `last` = the
// pixel's previous RGBD8 word, and two ping-pong planes of neighbour-update fire
// bits (one byte per pixel, bit j: channel j wrote into a neighbour at that frame;
// the neighbour and the slot follow from the pixel's Philox block 1 of that frame).
struct PbasConsts {
    int32_t N, min_matches;
    float R_incdec, R_scale, T_inc, T_dec, T_lower, T_upper;
    float R_lower[4];
    uint32_t depth_max_mm;
    uint32_t key0, key1;
    float grad_alpha;  // gradient-magnitude variant only
};

struct PbasPlanes {
    uint32_t* samples;
    uint32_t* dhist;
    float4* R;
    float4* T;
    uint2* S;
    uint32_t* last;
    uint8_t* fire[2];
    uint8_t* mask;
    // 1: the previous value lives in sample slot N (the first padding slot of the last
    // quad; set for N >= 33 not a multiple of 4) and `last` is unused; 0: in `last`.
    int32_t last_in_pad;
};

struct PbasStepArgs {
    PbasPlanes m;
    const uint8_t* rgb;
    const uint8_t* depth;
    int64_t rgb_stride, depth_stride;
    int32_t H, W, npix;
    int32_t depth_h, depth_w;  // 0: depth is H x W; else its size, upscaled to H x W
    uint32_t t;            // frame index
    int32_t apply_pending; // neighbour writes of frame t-1 (fire bytes) still to be applied
    int32_t streaming;     // 1: non-temporal sample traffic (working set beyond the last-level cache)
    PbasConsts c;
};

hipError_t pbas_launch_init_state(const PbasPlanes& m, int npix, const PbasConsts& c,
                                  hipStream_t s);
template <int NB>
struct PbasBatch {
    int32_t n;
    int32_t first[NB + 1];
    int32_t tiles_x[NB];
    PbasStepArgs a[NB];
};

hipError_t pbas_launch_step(const PbasStepArgs& a, hipStream_t s);
// One launch over n <= kBatchMax models past their fill frames with the same
// register class and cache policy (pbas_batch_key equal, not -1).
hipError_t pbas_launch_step_batch(const PbasStepArgs* a, int n, hipStream_t s);
int pbas_batch_key(const PbasStepArgs& a);  // -1: a fill frame (its own launch)
hipError_t pbas_launch_flush(const PbasPlanes& m, int H, int W, uint32_t t_prev, const PbasConsts& c,
                             hipStream_t s);
hipError_t pbas_launch_export(const PbasPlanes& m, int npix, int N, uint8_t* out, hipStream_t s);
hipError_t pbas_launch_import(const PbasPlanes& m, int npix, int N, const uint8_t* in,
                              hipStream_t s);

// ------------------------------------------- PBAS, gradient magnitudes ----
// The gradient-magnitude variant (pbas_grad_kernels.hip): slot k of pixel p is word
// k * npix + p of the plain slot planes `samples` (bytes R, G, B, depth code) and
// `gsamples` (colour magnitudes m_R, m_G, m_B, 0); D[k * npix + p] holds the four
// channels' d_min as float4, S their float sums; `last` and `last_g` the pixel's
// value and magnitudes of the previous frame (pending neighbour writes carry them);
// gsum[4 * (t mod 3) + j] the sum of frame t's colour magnitudes m_j (frame t adds
// into its slot, reads frame t-1's and clears frame t+1's).
struct PbasGradPlanes {
    uint32_t* samples;
    uint32_t* gsamples;
    float4* D;
    float4* R;
    float4* T;
    float4* S;
    uint32_t* last;
    uint32_t* last_g;
    uint8_t* fire[2];
    uint8_t* mask;
    unsigned long long* gsum;
};

struct PbasGradArgs {
    PbasGradPlanes m;
    const uint8_t* rgb;
    const uint8_t* depth;
    int64_t rgb_stride, depth_stride;
    int32_t H, W, npix;
    int32_t depth_h, depth_w;
    uint32_t t;
    int32_t apply_pending;
    PbasConsts c;
};

hipError_t pbas_grad_launch_init_state(const PbasGradPlanes& m, int npix, const PbasConsts& c, hipStream_t s);
// One frame: the fill kernel for t < N, else the tile step.
hipError_t pbas_grad_launch_step(const PbasGradArgs& a, hipStream_t s);
hipError_t pbas_grad_launch_flush(const PbasGradPlanes& m, int H, int W, uint32_t t_prev, const PbasConsts& c,
                                  hipStream_t s);
// Canonical payload (see include/fgs.h) <-> device layout; `t` = frames pushed.
hipError_t pbas_grad_launch_export(const PbasGradPlanes& m, int npix, int N, int64_t t, uint8_t* out,
                                   hipStream_t s);
hipError_t pbas_grad_launch_import(const PbasGradPlanes& m, int npix, int N, int64_t t, const uint8_t* in,
                                   hipStream_t s);

// ------------------------------------------------------------ serving ----
// One entry of a serving batch: the next frame of one stream.  GMM entries are
// cut into 256-pixel tiles, PBAS entries into 64x4 tiles (1-D 256-pixel tiles
// while the model is still filling its samples).
struct ServeEntry {
    int32_t algo;     // FGS_GMM or FGS_PBAS
    int32_t fill;     // PBAS frame < N
    int32_t tiles_x;  // PBAS tiles per row
    int32_t ntiles;
    GmmStepArgs g;
    PbasStepArgs p;
};
int serve_pbas_nmax(int N);  // register capacity class of a PBAS model
// One launch over every tile of every entry (prefix[i] = first tile of entry i,
// prefix[n] = total), grid-stride over a grid sized to the device.
hipError_t serve_launch(const ServeEntry* entries, const int32_t* prefix, int n, int total_tiles,
                        int gmm_K, int pbas_nmax, bool streaming, hipStream_t s);

// ---------------------------------------------------------- evaluation ----
// Device counters of the evaluation: kEvalSlots partial sums per count, count c
// (TP, TN, FP, FN) at acc[c * kEvalSlots ...]; the reader adds the slots.
constexpr int kEvalSlots = 64;
// acc += TP, TN, FP, FN of mask (rows W bytes apart) against gt.
hipError_t eval_launch_count(const uint8_t* mask, const uint8_t* gt, int64_t gt_stride, int H, int W,
                             unsigned long long* acc, hipStream_t s);
hipError_t eval_launch_zero(unsigned long long* acc, hipStream_t s);

// ------------------------------------------------------- static objects ----
// count[p] = mask[p] ? min(count[p] + 1, 65535) : 0; out[p] = count[p] >= M ? 255 : 0.
// count and out are 256-byte aligned planes of npix.
hipError_t static_launch_update(const uint8_t* mask, uint16_t* count, uint8_t* out, int64_t npix, uint32_t M,
                                hipStream_t s);
hipError_t static_launch_clear(uint16_t* count, uint8_t* out, int64_t npix, hipStream_t s);

// -------------------------------------------------------- diagnostics ----
hipError_t diag_launch_philox(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                              hipStream_t s);
hipError_t diag_launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t diag_launch_mix(void* planes, int64_t npix, int mode, hipStream_t s);

}  // namespace fgs
