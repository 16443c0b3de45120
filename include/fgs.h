/*
 * fgs.h -- C ABI of libfgs: RGB-D foreground segmentation (GMM and PBAS
 * background models) on AMD Instinct MI355X (gfx950).
 *
 * The library computes, for every pixel of every frame, the classify-and-
 * update step of the two RGB-D background models of Janus, Kryjak and Gorgon,
 * "Foreground object segmentation in RGB-D data implemented on GPU":
 *   - FGS_GMM:  a colour Gaussian mixture and a depth Gaussian mixture per
 *               pixel, combined into one decision (Sec. 3.1);
 *   - FGS_PBAS: a Pixel-Based Adaptive Segmenter whose samples carry RGB and
 *               depth, each component segmented and updated on its own
 *               (Sec. 3.2).
 * The host owns acquisition and allocates the model on the device; frames go
 * in, a binary mask comes out (Sec. 4.2).  Everything per pixel runs in the
 * library's own HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status: every function returns fgs_status; FGS_OK is 0.  Nothing aborts
 *    and nothing throws across this boundary.  fgs_last_error() returns a
 *    thread-local description of the last failure on the calling thread.
 *  - Images: RGB is interleaved 8-bit R,G,B; depth is uint16 millimetres with
 *    0 meaning "no depth".  Rows are addressed with a byte stride >= the
 *    packed row size.  Masks are uint8, 0 = background, 255 = foreground.
 *  - Memory: fgs_mem tells whether a caller pointer is host or device memory.
 *    The caller owns every buffer it passes; the library owns the model.
 *    Device pointers are read/written in the model's stream order.
 *  - Streams: a model runs on one HIP stream (hipStream_t passed as void*),
 *    either the caller's or, when NULL is passed, one the library creates at
 *    default priority.  A model is not thread-safe; distinct models are.
 *  - Device errors poison the model: later calls on it return FGS_ERR_DEVICE
 *    until fgs_destroy.
 */
#ifndef FGS_H
#define FGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGS_ABI_VERSION 6

typedef enum fgs_status {
    FGS_OK = 0,
    FGS_ERR_INVALID_ARG = 1,   /* bad pointer, size, stride, params or struct_size */
    FGS_ERR_OUT_OF_MEMORY = 2, /* device or pinned host allocation failed */
    FGS_ERR_DEVICE = 3,        /* a HIP call failed; the model is poisoned */
    FGS_ERR_BAD_STATE = 4,     /* call not valid in the model's current state */
    FGS_ERR_BUSY = 5,          /* resource temporarily unavailable */
    FGS_ERR_UNSUPPORTED = 6    /* valid request the library does not implement */
} fgs_status;

typedef enum fgs_algo { FGS_GMM = 1, FGS_PBAS = 2 } fgs_algo;

typedef enum fgs_mem { FGS_MEM_HOST = 0, FGS_MEM_DEVICE = 1 } fgs_mem;

typedef struct fgs_model fgs_model; /* opaque, owned by the library */

/*
 * GMM constants (Sec. 3.1).  Each pixel holds Kc colour Gaussians over (R,G,B)
 * and Kd depth Gaussians over the 8-bit depth code, each Gaussian a weight w,
 * a mean and one isotropic variance v.  Per frame, on the ranked pre-update
 * mixtures: q_k = |X - mu_k|^2 / v_k; the background set is the leading
 * Gaussians whose weights first sum past T_bg; delta_m = min q_k over it;
 * foreground iff Z = (delta_c - lambda^2) + w_depth*(delta_d - lambda^2) >= 0,
 * the depth term present only where depth > 0.  Update (Stauffer-Grimson):
 * first Gaussian with q < lambda^2 matches, w <- (1-alpha)w (+alpha if matched),
 * matched mean/variance move with rate rho (rho_mode), v >= v_min; no match replaces the
 * last Gaussian by (w_init, X, v_init); weights renormalised; ranked by
 * w/sqrt(v), stable, descending.  The depth model is updated only where
 * depth > 0.  Supported (Kc,Kd): (k,k) for k = 1..7, and (7,3).
 */
typedef struct fgs_gmm_params {
    uint32_t struct_size; /* = sizeof(fgs_gmm_params) */
    int32_t Kc, Kd;
    float alpha;          /* learning rate (weights; the mean/variance rate is rho_mode's) */
    float lambda;         /* match threshold in standard deviations */
    float T_bg;           /* background weight fraction */
    float w_init;         /* weight of a replacement Gaussian */
    float v_init_c, v_min_c; /* colour variance: new Gaussian, floor */
    float v_init_d, v_min_d; /* depth variance: new Gaussian, floor */
    float w_depth;        /* weight of the depth term in Z */
    int32_t depth_max_mm; /* depth full scale: code = floor((255*D + M/2)/M), >= 1 */
    int32_t rho_mode;     /* rate of the matched mean and variance: 0 rho = alpha;
                             1 rho = alpha / w, w the matched weight after its update and
                             before renormalisation (OpenCV's mixture rule, which Sec. 3.1
                             names as a basis); 2 rho = alpha * eta, eta = exp(-q/2) /
                             (2 pi v) the Eq. (1) density of the matched Gaussian at the
                             sample before its update (Stauffer-Grimson's rate; exp is not
                             correctly rounded, so results agree with other implementations
                             to rounding, not bit for bit) */
    int32_t decision;     /* 0: the Z rule above; 1: the literal Eq. (1) factors: per model
                             P_m = density_scale * exp(-delta_m/2) / (2 pi v), v the variance
                             of the background Gaussian attaining delta_m, P = P_c * P_d where
                             the depth term is present (else the single factor), foreground
                             iff P < density_threshold */
    float density_scale;  /* s of Sec. 3.1 (default 10000) */
    float density_threshold; /* decision 1 threshold (default 1) */
    int32_t var_mode;     /* 0: one variance per colour Gaussian; 1: one per colour channel:
                             q = sum_c (X_c - mu_c)^2 / v_c (squared Mahalanobis distance),
                             each channel's variance updated and floored on its own, new
                             Gaussians and floors at v_init_c / 3 and v_min_c / 3 per
                             channel, rank key w / sqrt(v_r + v_g + v_b) */
    /* Fields after depth_max_mm were appended: a caller passing an earlier struct
     * (struct_size 52: none of them; 56: rho_mode only; 68: up to density_threshold)
     * gets the defaults for the rest. */
} fgs_gmm_params;

/*
 * PBAS constants (Sec. 3.2).  Per pixel: N samples (32-bit words, bytes R, G,
 * B, depth code; depth code 0 = none recorded), and per channel j in
 * {R,G,B,D} a decision threshold R_j, an update rate T_j, the history D_j of N
 * minimal distances and its sum S_j.  The first N frames fill the samples.
 * Then per active channel (depth only where depth > 0): foreground iff fewer
 * than min_matches samples lie within R_j; a background channel replaces one
 * random sample (and its D slot) with probability 1/T_j and writes a random
 * 8-neighbour's own value into a random sample of that neighbour with
 * probability 1/T_j; R_j and T_j then adapt to d_bar = S_j/N within
 * [R_lower_j, inf) and [T_lower, T_upper].  Random words come from
 * Philox4x32-10 keyed by `seed` with counter (y*W + x, frame, call, 0).
 * Accepted: N in 2..64, min_matches in 1..N, R_lower_j > 0, 0 <= R_incdec < 1,
 * R_scale > 0, 0 < T_lower <= T_upper, T_inc > 0 and T_dec > 0 (T moves by
 * T_inc/d_bar or T_dec/d_bar, +-inf at d_bar = 0 before the clamp; a zero
 * increment would make that 0/0; a fixed update period is T_lower = T_upper),
 * gradient 0 or 1, grad_alpha >= 0 and finite.
 */
typedef struct fgs_pbas_params {
    uint32_t struct_size; /* = sizeof(fgs_pbas_params) */
    int32_t N;
    int32_t min_matches;
    float R_incdec, R_scale;
    float T_inc, T_dec, T_lower, T_upper;
    float R_lower[4];     /* per channel R, G, B, depth */
    int32_t depth_max_mm;
    int32_t gradient;     /* 0: the RGB-D samples of Sec. 3.2 (default).  1: the base
                             method's gradient-magnitude feature added to the colour
                             channels (opt-in; the paper's variant leaves it out): m_j =
                             (|gx| + |gy|) >> 3 of channel j's plane (3x3 Sobel, border
                             replicated), a sample slot holds (v, m) per colour channel,
                             dist = w_j * |m - B^m| + |v - B^v| in float32 with
                             w_j = grad_alpha / max(mean of m_j over the previous frame, 1),
                             D and S float32; the depth channel as in 0 */
    uint64_t seed;
    float grad_alpha;     /* gradient weight (default 10; >= 0, finite) */
    int32_t reserved1;    /* 0 */
    /* A caller passing the earlier 72-byte struct (no grad_alpha) gets its default. */
} fgs_pbas_params;

/* ABI version of the loaded library (FGS_ABI_VERSION it was built with). */
int32_t fgs_abi_version(void);

/* Static English name of a status code.  Never NULL. */
const char* fgs_status_str(fgs_status s);

/* Thread-local text of the last failure on this thread ("" if none).  The
 * pointer stays valid until the next fgs_* call on this thread. */
const char* fgs_last_error(void);

/* Fill *p with the default constants (the readings of Sec. 3.1 used by this
 * library: Kc = Kd = 3, alpha 0.01, lambda 2.5, T_bg 0.7, w_init 0.05,
 * v_init_c 675, v_min_c 12, v_init_d 25, v_min_d 1, w_depth 1, 10 m full scale,
 * rho_mode 0, decision 0, density_scale 10000, density_threshold 1, var_mode 0).
 * INVALID_ARG if p is NULL. */
fgs_status fgs_gmm_params_default(fgs_gmm_params* p);

/* Fill *p with the default PBAS constants (Sec. 3.2: N = 20; the rest from the
 * base method: min_matches 2, R_incdec 0.05, R_scale 5, T_inc 1, T_dec 0.05,
 * T in [2, 200], R_lower 18,18,18 and 4 for depth, 10 m full scale; gradient 0,
 * grad_alpha 10).
 * INVALID_ARG if p is NULL. */
fgs_status fgs_pbas_params_default(fgs_pbas_params* p);

/*
 * Create a model of `algo` for H x W frames (Sec. 4.2: the host allocates the
 * background model in device memory).  `params` points to fgs_gmm_params or
 * fgs_pbas_params matching `algo` (NULL = defaults).  `hip_stream` is the
 * hipStream_t to run on, or NULL for a library-owned stream.  On success *out
 * receives the model; its state is the fresh model (GMM: w = 0, mu = 0,
 * v = v_init; PBAS: empty samples, R = R_lower, T = T_lower, D = S = 0).
 * Errors: INVALID_ARG (H or W < 1, H*W > 2^28, bad params), OUT_OF_MEMORY,
 * DEVICE.  Uses the current HIP device.
 */
fgs_status fgs_create(fgs_algo algo, int32_t H, int32_t W, const void* params,
                      void* hip_stream, fgs_model** out);

/* Wait for the model's queued work, then free it.  NULL is accepted. */
fgs_status fgs_destroy(fgs_model* m);

/*
 * Run one classify-and-update step on the next frame (Sec. 3.1 / 3.2, one
 * launch per frame).  rgb: H rows of 3*W bytes at rgb_stride bytes apart;
 * depth: H rows of W uint16 at depth_stride bytes apart (both >= packed row
 * size).  where = FGS_MEM_HOST: the frame is copied to pinned staging and sent
 * to the device before return (the host buffers may be reused at once);
 * FGS_MEM_DEVICE: the kernel reads the device buffers in stream order, and the
 * caller must not overwrite them before the step has run (fgs_sync or a later
 * stream event).  Asynchronous otherwise: the mask is ready in stream order.
 * Errors: INVALID_ARG (NULL model or frame, a stride below the packed row, a
 * depth pointer or stride that is not 2-byte aligned, a bad `where`), BAD_STATE
 * (2^32 - 1 frames pushed: the PBAS random stream's frame counter is exhausted),
 * DEVICE (the model is then poisoned: every later call but fgs_destroy fails).
 */
fgs_status fgs_push_frame(fgs_model* m, const uint8_t* rgb, int64_t rgb_stride,
                          const uint16_t* depth, int64_t depth_stride, fgs_mem where);

/*
 * As fgs_push_frame, for a depth map of depth_H x depth_W pixels (depth_stride
 * bytes per row) taken at another resolution than the RGB frame: the kernel
 * brings it to the RGB grid by nearest-neighbour upscaling on pixel centres,
 * depth(x, y) = D[floor((y + 1/2) depth_H / H)][floor((x + 1/2) depth_W / W)]
 * (Sec. 4.3: depth is upscaled to the RGB resolution when they differ, e.g.
 * 1280x720 RGB with 848x480 depth).  With FGS_MEM_HOST the depth map may not
 * have more pixels than the RGB frame.  Errors as fgs_push_frame.
 */
fgs_status fgs_push_frame_scaled(fgs_model* m, const uint8_t* rgb, int64_t rgb_stride,
                                 const uint16_t* depth, int64_t depth_stride, int32_t depth_H,
                                 int32_t depth_W, fgs_mem where);

/*
 * Push one frame to each of n independent models (many cameras) with as few
 * launches as possible: the result is exactly that of fgs_push_frame(models[i],
 * rgb[i], rgb_stride[i], depth[i], depth_stride[i], FGS_MEM_DEVICE) for each i.
 * Models of one kind and class share a launch of up to 8 models (GMM: same Kc,
 * Kd, variant and cache policy; PBAS: past its N fill frames, same register class
 * of N and cache policy, not the gradient variant), so the device ramps up and
 * drains once per launch instead of once per model; other models get launches of
 * their own.
 *
 * Frames are device memory, each of its model's H x W size (no depth
 * upscaling), rows rgb_stride[i] >= 3W and depth_stride[i] >= 2W (even) bytes
 * apart, read in stream order as by fgs_push_frame.  Every model must have been
 * created on the same stream and device, and appear once.  1 <= n <= 4096.
 * Errors: INVALID_ARG for NULL arrays or entries, bad strides, mixed streams or
 * devices, a repeated model or n out of range; BAD_STATE for an exhausted frame
 * counter; DEVICE for a poisoned model.  These are checked for every model first,
 * and then no model takes its frame.  A failing launch poisons the models it
 * held and those whose launch had not been issued yet (DEVICE).
 */
fgs_status fgs_push_frames(fgs_model* const* models, int32_t n, const uint8_t* const* rgb,
                           const int64_t* rgb_stride, const uint16_t* const* depth,
                           const int64_t* depth_stride);

/*
 * Copy the mask of the most recent frame into `mask` (H rows of W bytes,
 * `stride` bytes apart; 255 = foreground, 0 = background).  FGS_MEM_HOST waits
 * for the frame to finish; FGS_MEM_DEVICE enqueues a device copy on the model's
 * stream.  Errors: INVALID_ARG (NULL, stride < W, bad `where`), BAD_STATE before
 * the first push, DEVICE.
 */
fgs_status fgs_get_mask(fgs_model* m, uint8_t* mask, int64_t stride, fgs_mem where);

/* Borrow the device pointer of the model's internal H*W mask buffer (valid
 * until fgs_destroy; rewritten by every push, in stream order).  INVALID_ARG
 * for NULL arguments. */
fgs_status fgs_mask_device_ptr(fgs_model* m, const uint8_t** out);

/*
 * Evaluation counters (Sec. 5).  The paper scores masks by PWC = 100 (FN + FP) /
 * (TP + TN + FP + FN), FNR = FN / (TP + FN), FPR = FP / (FP + TN) and
 * Si = TP / (TP + FP + FN), all functions of the confusion counts against a
 * ground-truth mask (foreground = positive).
 *
 * fgs_eval_accumulate compares the model's current mask with `gt` (H x W bytes,
 * nonzero = foreground, rows gt_stride >= W bytes apart, in host or device memory
 * per `where`) and adds TP, TN, FP, FN to a device-resident accumulator owned by
 * the model, on the model's stream, without waiting for the device.  A host gt is
 * copied to pinned staging before the call returns (the caller may reuse it); a
 * device gt is read in stream order.  The accumulator starts at zero.
 * INVALID_ARG for a NULL gt, a short stride or a bad `where`; BAD_STATE before the
 * first push (no mask yet).
 */
fgs_status fgs_eval_accumulate(fgs_model* m, const uint8_t* gt, int64_t gt_stride, fgs_mem where);

/* Wait for the model's stream and write the accumulated counts to counts[0..3] =
 * TP, TN, FP, FN (host memory; all zero if nothing was accumulated).  reset != 0
 * then clears the accumulator.  INVALID_ARG for NULL arguments, DEVICE. */
fgs_status fgs_eval_read(fgs_model* m, uint64_t counts[4], int32_t reset);


/*
 * Static-object detection on the model's masks.  The paper names the detection of
 * static objects as future work (Sec. 6) without a method; read here as: a pixel is
 * part of a static object once the mask has marked it foreground in each of the last M
 * frames.  Per pixel a run counter c = mask ? min(c + 1, 65535) : 0 is updated after
 * every push (fgs_push_frame, fgs_push_frame_scaled, fgs_push_frames; a kernel on the
 * model's stream reading the mask), and the static mask is 255 where c >= M, else 0.
 * The detector only reads the masks; the background model is not changed by it.
 *
 * fgs_static_enable: M in 1..65535 enables the detector (or restarts it with a new M)
 *   with every counter at 0, from the next push on (allocates 3 bytes per pixel of
 *   device memory on first use); M = 0 turns it off and frees them.  fgs_set_state
 *   restarts the counters.  Servers do not run it.  INVALID_ARG for M outside 0..65535,
 *   OUT_OF_MEMORY, DEVICE.
 * fgs_static_mask: copy the static mask after the last push (H rows of W bytes, stride
 *   bytes apart) to host memory (waits) or device memory (stream order).  BAD_STATE if
 *   the detector is off or has counted no frame yet; INVALID_ARG for NULL, stride < W
 *   or a bad `where`.
 */
fgs_status fgs_static_enable(fgs_model* m, int32_t M);
fgs_status fgs_static_mask(fgs_model* m, uint8_t* out, int64_t stride, fgs_mem where);

/*
 * Median post-filter of a binary mask.  The paper's method leaves its masks
 * unfiltered (Sec. 3); the base PBAS method it builds on smooths its output with a
 * median filter, and this call offers that step for any mask, e.g. the one
 * fgs_mask_device_ptr returns.
 *
 * dst(y, x) = 255 if more than half of the (2r+1) x (2r+1) pixels of src centred on
 * (y, x) are nonzero, else 0: the median of the window, reading a pixel as
 * background (0) or foreground (nonzero, taken as 255).  Window pixels outside
 * the image repeat the nearest edge pixel (replicated border), so every pixel,
 * edges included, sees (2r+1)^2 values.  radius 0 copies the mask as 0/255.
 *
 * src and dst are device buffers of H rows of W bytes, rows src_stride and
 * dst_stride >= W bytes apart; the caller owns both, and the byte ranges they
 * span must not overlap (the filter is not in place).  Runs on hip_stream (NULL:
 * the null stream) and returns after enqueueing: src is read and dst written in
 * stream order.  H = 0 or W = 0 is an empty image and enqueues nothing.
 * INVALID_ARG for NULL buffers of a nonempty image, H or W negative or above
 * 2^30, H * W above 2^34, a stride below W or above 2^32, radius outside 0..7,
 * or overlapping ranges; DEVICE if the launch fails.
 */
fgs_status fgs_mask_median(const uint8_t* src, int64_t src_stride, uint8_t* dst, int64_t dst_stride,
                           int32_t H, int32_t W, int32_t radius, void* hip_stream);

/*
 * Model state, serialised in a fixed layout (little-endian):
 *   header (64 bytes): uint32 magic 0x53534746 ("FGSS"), uint32 version (1),
 *     uint32 algo, int32 H, int32 W, int32 A, int32 B, int32 flags,
 *     int64 frames pushed, uint64 seed (PBAS, else 0), 16 bytes reserved.
 *     A,B = Kc,Kd (GMM) or N,0 (PBAS).  flags bit 0: GMM per-channel colour
 *     variances (var_mode 1); bit 1: PBAS gradient-magnitude samples (gradient 1);
 *     every other bit zero.
 *   GMM payload (float32 planes of H*W, row-major), in order:
 *     w_c[Kc], mu_c[Kc][3] (R,G,B), v_c[Kc] (v_c[Kc][3] with flags bit 0),
 *     w_d[Kd], mu_d[Kd], v_d[Kd] (each model's Gaussians in rank order).
 *   PBAS payload: samples[N] uint32 planes (bytes R,G,B,depth code),
 *     dhist[N] uint32 planes (bytes D_R, D_G, D_B, D_D), R[4] float32 planes,
 *     T[4] float32 planes, S[4] uint16 planes.
 *   PBAS payload with flags bit 1: samples[N] uint32 planes, gsamples[N] uint32
 *     planes (bytes m_R, m_G, m_B, 0), dhist[N][4] float32 planes (slot-major, then
 *     channel R, G, B, depth), R[4], T[4], S[4] float32 planes, then 3 uint64: the
 *     colour magnitude sums of the last frame pushed (the next frame's weights).
 * fgs_state_size gives the byte count.  fgs_copy_state first applies any
 * deferred PBAS neighbour writes (so the state is the logical model after the
 * last frame), then copies; FGS_MEM_HOST waits for completion.  fgs_set_state
 * replaces the model (including the frame counter, which keys the PBAS random
 * stream) from such a blob for the same algo/H/W/A/B.
 * A device buffer (FGS_MEM_DEVICE) must be 4-byte aligned.
 * Errors: INVALID_ARG (size or header mismatch, misaligned device buffer), DEVICE.
 */
fgs_status fgs_state_size(const fgs_model* m, size_t* bytes);
fgs_status fgs_copy_state(fgs_model* m, void* dst, size_t bytes, fgs_mem where);
fgs_status fgs_set_state(fgs_model* m, const void* src, size_t bytes, fgs_mem where);

/*
 * fgs_copy_state without allocating, for callers that cannot allocate device memory:
 * serving loops that checkpoint a camera's model between frames, harnesses that
 * forbid hipMalloc.  Same arguments, result and errors as fgs_copy_state, and the same
 * export kernels; a host destination is staged through a library-owned device buffer
 * of FGS_NOALLOC_STAGING_BYTES (64 MiB) instead of a buffer allocated for the call.
 * Each GPU the library runs on holds that buffer from the first call on it until the
 * process ends.  The call itself allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  Limit: a host copy's payload (fgs_state_size minus the
 * 64-byte header) must fit in the buffer, else UNSUPPORTED and nothing is copied; a
 * device destination needs no staging and has no limit.  All calls on one GPU share
 * its buffer, which keeps the last call's contents (every byte a call reads was written
 * by that call): calls that overlap on one GPU, from several threads or on several
 * streams, race, and the caller must serialise them.  The call waits for its stream,
 * so it cannot be recorded into a HIP graph.
 * Errors: INVALID_ARG, UNSUPPORTED (payload beyond the buffer), DEVICE.
 */
#define FGS_NOALLOC_STAGING_BYTES ((size_t)64 << 20)
fgs_status fgs_copy_state_noalloc(fgs_model* m, void* dst, size_t bytes, fgs_mem where);

/*
 * In-place access to the model's device state (Sec. 3.1, 3.2: the per-pixel model
 * the host allocated on the device, Sec. 4.2), for callers that read it where it
 * lives instead of copying it.  Each field is one per-pixel value: element p (the
 * pixel y*W + x) of field f is at (const char*)f.base + p * f.pixel_stride, of type
 * f.dtype.  Fields come in the serialised payload's order:
 *   GMM:  w_c[k], mu_c[k][c], v_c[k] (v_c[k][c] with var_mode 1), w_d[k], mu_d[k],
 *         v_d[k]; float32.
 *   PBAS: samples[k] and dhist[k] uint32 (bytes R,G,B,depth), R[j], T[j] float32,
 *         S[j] uint16; with gradient 1: samples[k], gsamples[k] uint32, dhist[k][j],
 *         R[j], T[j], S[j] float32.
 * `name` is a static string naming the array, `index` the rank, slot or channel,
 * `sub` the colour channel of mu_c and per-channel v_c (else 0).
 * With fields == NULL (capacity ignored) the call only writes the number of fields
 * to *count.  Otherwise capacity must be at least that number; a PBAS model first
 * applies the neighbour writes still deferred from its last frame, on its stream,
 * so that the fields hold the logical state after the last frame once the stream
 * has reached this call (fgs_sync, or a wait on fgs_stream's stream).
 * The addresses are borrowed: they stay valid until fgs_destroy; the next push or
 * fgs_set_state changes what they hold.  Writing through them is not supported.
 * Errors: INVALID_ARG (NULL count, capacity too small), DEVICE.
 */
typedef enum fgs_dtype { FGS_DTYPE_F32 = 1, FGS_DTYPE_U32 = 2, FGS_DTYPE_U16 = 3 } fgs_dtype;
typedef struct fgs_state_field {
    const char* name;
    int32_t index;
    int32_t sub;
    int32_t dtype;        /* fgs_dtype */
    int32_t elem_bytes;
    const void* base;     /* device address of pixel 0's element */
    int64_t pixel_stride; /* bytes from one pixel's element to the next pixel's */
} fgs_state_field;
fgs_status fgs_get_state(fgs_model* m, fgs_state_field* fields, int32_t capacity, int32_t* count);

/* Number of frames pushed so far (the next frame's index; it keys the PBAS
 * random stream, Sec. 3.2).  INVALID_ARG for NULL arguments. */
fgs_status fgs_frame_index(const fgs_model* m, int64_t* t);

/* Block until all work queued on the model's stream has finished.  INVALID_ARG
 * for NULL, DEVICE if that work failed. */
fgs_status fgs_sync(fgs_model* m);

/* The hipStream_t (as void*) the model runs on (owned by the library unless the
 * caller passed one to fgs_create).  INVALID_ARG for NULL arguments. */
fgs_status fgs_stream(const fgs_model* m, void** hip_stream);

/* Device bytes the model holds (state, scratch planes, mask, input staging).
 * INVALID_ARG for NULL arguments. */
fgs_status fgs_device_bytes(const fgs_model* m, size_t* bytes);

/*
 * How the model's per-frame state traffic treats the last-level (Infinity)
 * cache.  The state is read and written once per frame, so it is either kept
 * cache-resident between frames (worth it while all live models fit) or
 * streamed with non-temporal accesses.  FGS_CACHE_AUTO (default) streams once
 * the device bytes of all live models on the device exceed the threshold
 * FGS_STREAMING_THRESHOLD_MB (environment, default 192).  Results are identical
 * under every policy.  INVALID_ARG for an unknown policy.
 */
typedef enum fgs_cache_policy { FGS_CACHE_AUTO = 0, FGS_CACHE_KEEP = 1, FGS_CACHE_STREAM = 2 } fgs_cache_policy;
fgs_status fgs_set_cache_policy(fgs_model* m, int32_t policy);

/*
 * GMM adjoint over a window of frames (gradient of a loss on the pre-update scores
 * with respect to theta = (alpha, lambda, w_depth)).
 *
 * The window starts from a fresh GMM (Sec. 3.1; constants other than theta from
 * `params`, which must have Kc == Kd in 1..5) and runs T frames.  Frame t yields
 * the score Z_t = (delta_c - lambda^2) + w_depth*(delta_d - lambda^2) of the
 * pre-update model (terms only where the model has data, depth only where
 * D > 0; Z_t = 0 and has_term = 0 where neither exists) -- the quantity the mask
 * thresholds at zero.  fgs_gmm_window_forward records the discrete choices of
 * every step (background Gaussian attaining delta, matched Gaussian or
 * replacement, variance floor, ranking) and checkpoints the means and variances
 * every `checkpoint_every` frames.  fgs_gmm_window_backward holds those choices
 * fixed and returns dtheta[i] = sum over t, pixels of dZ[t] * dZ_t/dtheta_i,
 * replaying each segment from its checkpoint; the sum is reduced in a fixed
 * order (deterministic).
 *
 * All arrays are device memory, dense, in the window's stream order:
 * theta float[3]; rgb uint8[T][H][W][3]; depth uint16[T][H][W]; Z float[T][H][W];
 * has_term uint8[T][H][W]; dZ float[T][H][W]; dtheta double[3].  A window holds the
 * records and checkpoints of its most recent forward only: backward differentiates that
 * forward, so it must be given the same theta and frames, unchanged since (a caller that
 * runs several forwards on one window reruns the one it differentiates first).  `hip_stream` as in
 * fgs_create.  Errors: INVALID_ARG, UNSUPPORTED (K, or rho_mode, decision or var_mode
 * != 0: the adjoint is derived for rho = alpha, the Z score and one variance per
 * Gaussian), OUT_OF_MEMORY, BAD_STATE
 * (backward or records before forward), DEVICE.
 */
typedef struct fgs_gmm_window fgs_gmm_window;
fgs_status fgs_gmm_window_create(int32_t T, int32_t H, int32_t W, const fgs_gmm_params* params,
                                 int32_t checkpoint_every, void* hip_stream, fgs_gmm_window** out);
fgs_status fgs_gmm_window_forward(fgs_gmm_window* w, const float* theta, const uint8_t* rgb,
                                  const uint16_t* depth, float* Z, uint8_t* has_term);
fgs_status fgs_gmm_window_backward(fgs_gmm_window* w, const float* theta, const uint8_t* rgb,
                                   const uint16_t* depth, const float* dZ, double* dtheta);
/* Copy the last forward's records (uint64[T][H][W], layout documented in the
 * library source) to host or device memory. */
fgs_status fgs_gmm_window_records(fgs_gmm_window* w, uint64_t* out, fgs_mem where);
fgs_status fgs_gmm_window_destroy(fgs_gmm_window* w);

/*
 * Multi-stream serving.  Many camera streams on one GPU, every model resident in
 * device memory, frames batched continuously: a scheduler thread takes the next
 * queued frame of every stream whose previous frame has finished (at most one
 * frame per stream in flight, so each stream's frames run in order), copies the
 * inputs over, runs them on the device and copies the masks back, without waiting
 * for earlier batches; a completion thread stamps each frame's latency.  Per-stream
 * results are exactly those of a model driven alone with fgs_push_frame.
 * Within a batch, GMM streams with Kc = Kd = K (K = 3 or 5, one variance per
 * Gaussian, any rate or decision variant) and PBAS streams with N <= 40 run in ONE
 * launch of the serving kernel (mixed resolutions, GMM and PBAS; for the K, whichever
 * of 3 and 5 has more of the batch's pixels); every other stream runs in the
 * per-frame step kernels, models of one kernel class sharing a launch of up to 8,
 * after it on the same stream.
 *
 * fgs_server_create: `hbm_budget_bytes` caps the device memory of all open
 *   streams (models, input slots) plus the server's own buffers; up to
 *   `max_streams` (1..1024) streams.  Uses the current device.
 * fgs_server_open: admit a stream with any params fgs_create accepts (errors as
 *   fgs_create).  BUSY when the budget or the stream slots would be exceeded, also
 *   between opens that run concurrently (nothing stays allocated then).
 * fgs_server_submit: copy one host frame (dense rgb uint8[H][W][3], depth
 *   uint16[H][W]) into the stream's ring (4 frames) and return a ticket; the
 *   buffers may be reused at once.  t_arrival_s is the frame's arrival on the
 *   fgs_server_now() clock (<= 0: now).  BUSY when 4 frames of the stream are
 *   pending or uncollected.
 * fgs_server_wait: block until the ticket's frame is done (timeout_ms < 0:
 *   forever; else BUSY on timeout), copy its mask (host uint8[H][W]; NULL to
 *   skip), report its latency (completion - arrival, seconds) and release the
 *   slot.  BAD_STATE if the frame was dropped by fgs_server_close, DEVICE after
 *   a device error.  A ticket is collected once: INVALID_ARG for a ticket that
 *   was never issued or that another wait already collected (also when that
 *   wait ran concurrently).
 * fgs_server_close: stop a stream; its frame in flight finishes, queued frames
 *   are dropped, its device memory returns to the budget, and its pinned host
 *   ring is freed once its last ticket is collected.
 * fgs_server_get_stats: since creation or the last fgs_server_reset_stats:
 *   completed frames, batches, mean frames per batch, p50 / p99 / max latency,
 *   completed pixel-frames per second, budget use.  Set struct_size first.
 * fgs_server_destroy: finish the batches in flight and free everything; no other
 *   call on the server may run concurrently with it.
 * All other server calls are thread-safe.
 */
typedef struct fgs_server fgs_server;
typedef struct fgs_server_stats {
    uint32_t struct_size; /* = sizeof(fgs_server_stats) */
    int32_t streams_open;
    int64_t frames_done;
    int64_t batches;
    double mean_batch_frames;
    double p50_latency_s, p99_latency_s, max_latency_s;
    double mpix_frames_per_s;
    uint64_t device_bytes_used, device_budget;
} fgs_server_stats;
double fgs_server_now(void);
fgs_status fgs_server_create(size_t hbm_budget_bytes, int32_t max_streams, fgs_server** out);
fgs_status fgs_server_open(fgs_server* s, fgs_algo algo, int32_t H, int32_t W, const void* params,
                           int32_t* stream_id);
fgs_status fgs_server_submit(fgs_server* s, int32_t stream_id, const uint8_t* rgb,
                             const uint16_t* depth, double t_arrival_s, uint64_t* ticket);
fgs_status fgs_server_wait(fgs_server* s, uint64_t ticket, uint8_t* mask, double* latency_s,
                           int32_t timeout_ms);
fgs_status fgs_server_close(fgs_server* s, int32_t stream_id);
fgs_status fgs_server_get_stats(fgs_server* s, fgs_server_stats* out);
fgs_status fgs_server_reset_stats(fgs_server* s);
fgs_status fgs_server_destroy(fgs_server* s);

/*
 * Diagnostics.
 * fgs_philox4x32_10: for i < n, out[4i..4i+3] = Philox4x32-10(ctr[4i..4i+3],
 *   key = (seed low 32 bits, seed high 32 bits)) (Salmon et al., SC'11) -- the
 *   generator PBAS draws from.  ctr and out are device arrays of 4n uint32;
 *   runs on hip_stream (NULL = default stream) and returns after enqueueing.
 * fgs_copy_probe: a plain streaming device copy of `bytes` (multiple of 16,
 *   both pointers 16-byte aligned) used to calibrate achievable HBM bandwidth.
 * fgs_mix_probe: the step kernels' access shape without their arithmetic, to
 *   calibrate what HBM gives a read/write mix: one lane per pixel over float4
 *   planes of npix pixels at `planes` (device, 16-byte aligned, at least 10 planes,
 *   i.e. 160*npix bytes, which it overwrites), non-temporal accesses.  mode 0: read
 *   10 planes, write all 10 back in place; 1: read 10, write the first 5 back
 *   (about GMM K=5's mix); 2: read 10 only; 3: write 10 only; 4: read 9, write 9
 *   back (PBAS N=35's sample quads).  Runs on hip_stream, returns after enqueueing.
 *   INVALID_ARG for a bad buffer, npix or mode.
 */
fgs_status fgs_philox4x32_10(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                             void* hip_stream);
fgs_status fgs_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream);
fgs_status fgs_mix_probe(void* planes, int64_t npix, int32_t mode, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FGS_H */
