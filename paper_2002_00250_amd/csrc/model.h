// Internal: the model object behind fgs_model* and the host-side preparation of
// one frame's launch arguments, shared by fgs_push_frame and the server.
#pragma once

#include <hip/hip_runtime.h>

#include "fgs.h"
#include "fgs_internal.h"

struct fgs_model {
    fgs_algo algo;
    int32_t H, W, npix;
    fgs_gmm_params gp;
    fgs_pbas_params pp;
    fgs::GmmConsts gc;
    fgs::PbasConsts pc;
    int device;
    hipStream_t stream;
    bool own_stream;
    uint8_t* dev;      // one allocation: state + scratch planes + mask
    size_t dev_bytes;
    float4* gmm_state;
    fgs::PbasPlanes pb;
    fgs::PbasGradPlanes pg;  // PBAS with the gradient-magnitude feature (pp.gradient)
    uint8_t* mask;
    // host-frame staging (allocated on the first host push)
    uint8_t* host_stage;
    uint8_t* dev_in;
    hipEvent_t stage_done;
    bool stage_busy;
    // evaluation (allocated on the first fgs_eval_accumulate)
    unsigned long long* eval_acc;  // device: TP, TN, FP, FN, kEvalSlots partial sums each
    uint8_t* gt_stage;             // pinned host copy of a host ground truth
    uint8_t* gt_dev;               // its device copy
    hipEvent_t gt_done;
    bool gt_busy;
    // static-object detection (fgs_static_enable): run counters and the static mask
    uint16_t* st_count;
    uint8_t* st_mask;
    int32_t st_M;       // 0: off
    int64_t st_frames;  // frames counted since the detector was enabled
    int64_t t;          // frames pushed
    bool pending;       // PBAS: neighbour writes of frame t-1 not yet applied
    bool poisoned;
    int32_t cache_policy;  // fgs_cache_policy
};

namespace fgs {

// Thread-local error text + status (fgs_last_error).
fgs_status set_error(fgs_status s, const char* fmt, ...);
// GMM parameters from a caller's struct (NULL: defaults), honouring struct_size: the
// current layout, or the earlier one without rho_mode (which then defaults to 0).
fgs_status load_gmm_params(const void* src, fgs_gmm_params* out);
// Launch constants of checked GMM parameters.
GmmConsts gmm_consts(const fgs_gmm_params& p);
// Non-temporal state traffic for this model's next launch (cache policy).
bool model_use_streaming(const fgs_model* m);
// Launch arguments of the model's next frame read from device frames; advances the
// model's frame counter and pending-write flag exactly as a push does.
// depth_h = depth_w = 0: the depth map has the model's size.
void model_next_gmm(fgs_model* m, const uint8_t* rgb, int64_t rgb_stride, const uint8_t* depth,
                    int64_t depth_stride, int32_t depth_h, int32_t depth_w, GmmStepArgs* a);
void model_next_pbas(fgs_model* m, const uint8_t* rgb, int64_t rgb_stride, const uint8_t* depth,
                     int64_t depth_stride, int32_t depth_h, int32_t depth_w, PbasStepArgs* a);
void model_next_pbas_grad(fgs_model* m, const uint8_t* rgb, int64_t rgb_stride, const uint8_t* depth,
                          int64_t depth_stride, int32_t depth_h, int32_t depth_w, PbasGradArgs* a);
// PBAS parameters from a caller's struct (NULL: defaults), honouring struct_size: the
// current layout, or the earlier one without grad_alpha (which then defaults).
fgs_status load_pbas_params(const void* src, fgs_pbas_params* out);

}  // namespace fgs
