// libfgs runtime: the C ABI of include/fgs.h.  Owns model objects, their device
// memory (one allocation per model, every plane 256-byte aligned), the pinned
// staging used for host frames, and the stream each model runs on.  All
// per-pixel work is done by the kernels in gmm_kernels.hip / pbas_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fgs.h"
#include "fgs_internal.h"
#include "model.h"
#include "postfilter.h"

using namespace fgs;

// The staging buffer of fgs_copy_state_noalloc (see noalloc_staging below).
static __device__ __align__(256) uint8_t scratch[FGS_NOALLOC_STAGING_BYTES];

namespace {

thread_local std::string g_last_error;

}  // namespace

fgs_status fgs::set_error(fgs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

namespace {

template <typename... A>
fgs_status fail(fgs_status s, const char* fmt, A... args) {
    return fgs::set_error(s, fmt, args...);
}

constexpr uint32_t kStateMagic = 0x53534746u;  // "FGSS"
constexpr uint32_t kStateVersion = 1;
constexpr size_t kHeaderBytes = 64;
constexpr int64_t kMaxPixels = int64_t(1) << 28;

struct StateHeader {
    uint32_t magic, version, algo;
    int32_t H, W, A, B, flags;  // flags bit 0: per-channel colour variances (GMM)
    int64_t frames;
    uint64_t seed;
    uint8_t pad[16];
};
static_assert(sizeof(StateHeader) == kHeaderBytes, "state header is 64 bytes");

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Device bytes held by live models, per device: the kernels stream state with
// non-temporal accesses once this exceeds what the last-level cache can keep.
constexpr int kMaxDevices = 64;
constexpr size_t kNoallocBytes = FGS_NOALLOC_STAGING_BYTES;
std::atomic<int64_t> g_resident[kMaxDevices];

int64_t streaming_threshold() {
    static const int64_t v = [] {
        const char* e = std::getenv("FGS_STREAMING_THRESHOLD_MB");
        const long long mb = e ? std::atoll(e) : 192;  // below the 256 MB Infinity Cache
        return (int64_t)mb << 20;
    }();
    return v;
}

}  // namespace



namespace {

fgs_status device_fail(fgs_model* m, hipError_t e, const char* what) {
    if (m) m->poisoned = true;
    return fail(FGS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define FGS_HIP(m, call)                                         \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return device_fail((m), e_, #call); \
    } while (0)

size_t gmm_payload_bytes(const fgs_model* m) {
    return (size_t)((m->gp.var_mode ? 7 : 5) * m->gp.Kc + 3 * m->gp.Kd) * (size_t)m->npix * 4;
}
size_t pbas_payload_bytes(const fgs_model* m) {
    const size_t n = (size_t)m->npix;
    if (m->pp.gradient) return (6 * (size_t)m->pp.N + 12) * n * 4 + 3 * 8;
    return 2 * (size_t)m->pp.N * n * 4 + 8 * n * 4 + 4 * n * 2;
}
size_t payload_bytes(const fgs_model* m) {
    return m->algo == FGS_GMM ? gmm_payload_bytes(m) : pbas_payload_bytes(m);
}

fgs_status check_gmm(const fgs_gmm_params& p) {
    if (p.struct_size != sizeof(fgs_gmm_params))
        return fail(FGS_ERR_INVALID_ARG, "fgs_gmm_params.struct_size %u != %zu", p.struct_size,
                    sizeof(fgs_gmm_params));
    if (p.rho_mode < 0 || p.rho_mode > 2) return fail(FGS_ERR_INVALID_ARG, "rho_mode %d not 0, 1 or 2", p.rho_mode);
    if (p.decision != 0 && p.decision != 1) return fail(FGS_ERR_INVALID_ARG, "decision %d not 0 or 1", p.decision);
    if (p.var_mode != 0 && p.var_mode != 1) return fail(FGS_ERR_INVALID_ARG, "var_mode %d not 0 or 1", p.var_mode);
    if (!(p.density_scale > 0.f && p.density_scale < INFINITY) ||
        !(p.density_threshold >= 0.f && p.density_threshold < INFINITY))
        return fail(FGS_ERR_INVALID_ARG, "density_scale must be > 0 and density_threshold >= 0, both finite");
    if (!gmm_supported(p.Kc, p.Kd))
        return fail(FGS_ERR_INVALID_ARG, "unsupported (Kc, Kd) = (%d, %d)", p.Kc, p.Kd);
    if (!(p.alpha > 0.f && p.alpha < 1.f) || !(p.lambda > 0.f) || !(p.T_bg > 0.f && p.T_bg < 1.f) ||
        !(p.w_init > 0.f) || !(p.v_min_c > 0.f) || !(p.v_init_c >= p.v_min_c) ||
        !(p.v_min_d > 0.f) || !(p.v_init_d >= p.v_min_d) || !(p.w_depth >= 0.f) ||
        p.depth_max_mm < 1)
        return fail(FGS_ERR_INVALID_ARG, "GMM parameter out of range");
    return FGS_OK;
}

fgs_status check_pbas(const fgs_pbas_params& p) {
    if (p.struct_size != sizeof(fgs_pbas_params))
        return fail(FGS_ERR_INVALID_ARG, "fgs_pbas_params.struct_size %u != %zu", p.struct_size,
                    sizeof(fgs_pbas_params));
    if (p.N < 2 || p.N > 64) return fail(FGS_ERR_INVALID_ARG, "PBAS N = %d not in [2, 64]", p.N);
    if (p.gradient != 0 && p.gradient != 1) return fail(FGS_ERR_INVALID_ARG, "gradient %d not 0 or 1", p.gradient);
    if (!(p.grad_alpha >= 0.f && p.grad_alpha < INFINITY) || p.reserved1 != 0)
        return fail(FGS_ERR_INVALID_ARG, "grad_alpha must be >= 0 and finite, reserved1 0");
    if (p.min_matches < 1 || p.min_matches > p.N)
        return fail(FGS_ERR_INVALID_ARG, "min_matches = %d not in [1, N]", p.min_matches);
    if (!(p.T_lower > 0.f) || !(p.T_upper >= p.T_lower) || !(p.R_scale > 0.f) ||
        !(p.R_incdec >= 0.f && p.R_incdec < 1.f) || !(p.T_inc > 0.f) || !(p.T_dec > 0.f) ||
        p.depth_max_mm < 1)
        return fail(FGS_ERR_INVALID_ARG, "PBAS parameter out of range");
    for (int j = 0; j < 4; ++j)
        if (!(p.R_lower[j] > 0.f)) return fail(FGS_ERR_INVALID_ARG, "R_lower[%d] must be > 0", j);
    return FGS_OK;
}

fgs_status ensure_staging(fgs_model* m) {
    if (m->host_stage) return FGS_OK;
    const size_t bytes = align256((size_t)m->npix * 3) + align256((size_t)m->npix * 2);
    hipError_t e = hipHostMalloc((void**)&m->host_stage, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        m->host_stage = nullptr;
        return fail(FGS_ERR_OUT_OF_MEMORY, "pinned staging of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    e = hipMalloc((void**)&m->dev_in, bytes);
    if (e != hipSuccess) {
        (void)hipHostFree(m->host_stage);
        m->host_stage = nullptr;
        m->dev_in = nullptr;
        return fail(FGS_ERR_OUT_OF_MEMORY, "device input staging of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    FGS_HIP(m, hipEventCreateWithFlags(&m->stage_done, hipEventDisableTiming));
    m->stage_busy = false;
    return FGS_OK;
}

}  // namespace

fgs_status fgs::load_gmm_params(const void* src, fgs_gmm_params* p) {
    fgs_gmm_params_default(p);
    if (!src) return FGS_OK;
    // earlier layouts: up to depth_max_mm, then with rho_mode, then up to density_threshold
    constexpr size_t kV1 = offsetof(fgs_gmm_params, rho_mode);
    constexpr size_t kV2 = offsetof(fgs_gmm_params, decision);
    constexpr size_t kV3 = offsetof(fgs_gmm_params, var_mode);
    uint32_t size = 0;
    std::memcpy(&size, src, sizeof size);
    if (size != sizeof(fgs_gmm_params) && size != kV1 && size != kV2 && size != kV3)
        return fail(FGS_ERR_INVALID_ARG, "fgs_gmm_params.struct_size %u is none of %zu, %zu, %zu, %zu", size,
                    sizeof(fgs_gmm_params), kV3, kV2, kV1);
    std::memcpy(p, src, size);  // the fields it does not cover keep their defaults
    p->struct_size = sizeof *p;
    return FGS_OK;
}

fgs_status fgs::load_pbas_params(const void* src, fgs_pbas_params* p) {
    fgs_pbas_params_default(p);
    if (!src) return FGS_OK;
    constexpr size_t kV1 = offsetof(fgs_pbas_params, grad_alpha);  // the layout before grad_alpha
    uint32_t size = 0;
    std::memcpy(&size, src, sizeof size);
    if (size != sizeof(fgs_pbas_params) && size != kV1)
        return fail(FGS_ERR_INVALID_ARG, "fgs_pbas_params.struct_size %u is neither %zu nor %zu", size,
                    sizeof(fgs_pbas_params), kV1);
    std::memcpy(p, src, size);  // the fields it does not cover keep their defaults
    p->struct_size = sizeof *p;
    return FGS_OK;
}

GmmConsts fgs::gmm_consts(const fgs_gmm_params& p) {
    // per-channel colour variances start and are floored at a third of the isotropic
    // constants (the isotropic variance is the sum of the three)
    const float vi = p.var_mode ? p.v_init_c / 3.0f : p.v_init_c;
    const float vm = p.var_mode ? p.v_min_c / 3.0f : p.v_min_c;
    return GmmConsts{p.alpha, p.lambda,   p.T_bg,    p.w_init,
                     vi,      vm,         p.v_init_d, p.v_min_d,
                     p.w_depth, (uint32_t)p.depth_max_mm, p.rho_mode,
                     p.decision == 1 ? 1 : 0, p.density_scale, p.density_threshold, p.var_mode};
}

bool fgs::model_use_streaming(const fgs_model* m) {
    if (m->cache_policy == FGS_CACHE_STREAM) return true;
    if (m->cache_policy == FGS_CACHE_KEEP) return false;
    const int d = m->device >= 0 && m->device < kMaxDevices ? m->device : 0;
    return g_resident[d].load(std::memory_order_relaxed) > streaming_threshold();
}

void fgs::model_next_gmm(fgs_model* m, const uint8_t* rgb, int64_t rs, const uint8_t* depth, int64_t ds,
                         int32_t dh, int32_t dw, GmmStepArgs* a) {
    a->depth_h = dh;
    a->depth_w = dw;
    a->state = m->gmm_state;
    a->mask = m->mask;
    a->rgb = rgb;
    a->depth = depth;
    a->rgb_stride = rs;
    a->depth_stride = ds;
    a->H = m->H;
    a->W = m->W;
    a->npix = m->npix;
    a->streaming = model_use_streaming(m) ? 1 : 0;
    a->c = m->gc;
    m->t += 1;
}

void fgs::model_next_pbas(fgs_model* m, const uint8_t* rgb, int64_t rs, const uint8_t* depth, int64_t ds,
                          int32_t dh, int32_t dw, PbasStepArgs* a) {
    a->depth_h = dh;
    a->depth_w = dw;
    a->m = m->pb;
    a->rgb = rgb;
    a->depth = depth;
    a->rgb_stride = rs;
    a->depth_stride = ds;
    a->H = m->H;
    a->W = m->W;
    a->npix = m->npix;
    a->t = (uint32_t)m->t;
    a->apply_pending = m->pending ? 1 : 0;
    a->streaming = model_use_streaming(m) ? 1 : 0;
    a->c = m->pc;
    m->pending = m->t >= m->pp.N;
    m->t += 1;
}

void fgs::model_next_pbas_grad(fgs_model* m, const uint8_t* rgb, int64_t rs, const uint8_t* depth, int64_t ds,
                               int32_t dh, int32_t dw, PbasGradArgs* a) {
    a->depth_h = dh;
    a->depth_w = dw;
    a->m = m->pg;
    a->rgb = rgb;
    a->depth = depth;
    a->rgb_stride = rs;
    a->depth_stride = ds;
    a->H = m->H;
    a->W = m->W;
    a->npix = m->npix;
    a->t = (uint32_t)m->t;
    a->apply_pending = m->pending ? 1 : 0;
    a->c = m->pc;
    m->pending = m->t >= m->pp.N;
    m->t += 1;
}

namespace {

// The static-object detector counts the frame just pushed (on the model's stream).
fgs_status static_after_push(fgs_model* m) {
    if (m->st_M <= 0) return FGS_OK;
    FGS_HIP(m, static_launch_update(m->mask, m->st_count, m->st_mask, m->npix, (uint32_t)m->st_M, m->stream));
    m->st_frames += 1;
    return FGS_OK;
}

fgs_status flush_pending(fgs_model* m) {
    if (m->algo != FGS_PBAS || !m->pending) return FGS_OK;
    if (m->pp.gradient)
        FGS_HIP(m, pbas_grad_launch_flush(m->pg, m->H, m->W, (uint32_t)(m->t - 1), m->pc, m->stream));
    else
        FGS_HIP(m, pbas_launch_flush(m->pb, m->H, m->W, (uint32_t)(m->t - 1), m->pc, m->stream));
    m->pending = false;
    return FGS_OK;
}

}  // namespace

extern "C" {

int32_t fgs_abi_version(void) { return FGS_ABI_VERSION; }

const char* fgs_status_str(fgs_status s) {
    switch (s) {
        case FGS_OK: return "ok";
        case FGS_ERR_INVALID_ARG: return "invalid argument";
        case FGS_ERR_OUT_OF_MEMORY: return "out of memory";
        case FGS_ERR_DEVICE: return "device error";
        case FGS_ERR_BAD_STATE: return "bad state";
        case FGS_ERR_BUSY: return "busy";
        case FGS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* fgs_last_error(void) { return g_last_error.c_str(); }

fgs_status fgs_gmm_params_default(fgs_gmm_params* p) {
    if (!p) return fail(FGS_ERR_INVALID_ARG, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof *p;
    p->Kc = 3;
    p->Kd = 3;
    p->alpha = 0.01f;
    p->lambda = 2.5f;
    p->T_bg = 0.7f;
    p->w_init = 0.05f;
    p->v_init_c = 675.0f;
    p->v_min_c = 12.0f;
    p->v_init_d = 25.0f;
    p->v_min_d = 1.0f;
    p->w_depth = 1.0f;
    p->depth_max_mm = 10000;
    p->rho_mode = 0;
    p->decision = 0;
    p->density_scale = 10000.0f;
    p->density_threshold = 1.0f;
    p->var_mode = 0;
    return FGS_OK;
}

fgs_status fgs_pbas_params_default(fgs_pbas_params* p) {
    if (!p) return fail(FGS_ERR_INVALID_ARG, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->struct_size = sizeof *p;
    p->N = 20;
    p->min_matches = 2;
    p->R_incdec = 0.05f;
    p->R_scale = 5.0f;
    p->T_inc = 1.0f;
    p->T_dec = 0.05f;
    p->T_lower = 2.0f;
    p->T_upper = 200.0f;
    p->R_lower[0] = p->R_lower[1] = p->R_lower[2] = 18.0f;
    p->R_lower[3] = 4.0f;
    p->depth_max_mm = 10000;
    p->seed = 0x200200250ull;
    p->gradient = 0;
    p->grad_alpha = 10.0f;
    p->reserved1 = 0;
    return FGS_OK;
}

fgs_status fgs_create(fgs_algo algo, int32_t H, int32_t W, const void* params, void* hip_stream,
                      fgs_model** out) {
    if (!out) return fail(FGS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (algo != FGS_GMM && algo != FGS_PBAS) return fail(FGS_ERR_INVALID_ARG, "unknown algo %d", (int)algo);
    if (H < 1 || W < 1 || (int64_t)H * W > kMaxPixels)
        return fail(FGS_ERR_INVALID_ARG, "bad frame size %d x %d", H, W);

    fgs_model* m = new (std::nothrow) fgs_model();
    if (!m) return fail(FGS_ERR_OUT_OF_MEMORY, "host allocation");
    m->algo = algo;
    m->H = H;
    m->W = W;
    m->npix = H * W;
    fgs_gmm_params_default(&m->gp);
    fgs_pbas_params_default(&m->pp);
    fgs_status st = FGS_OK;
    if (algo == FGS_GMM) {
        st = load_gmm_params(params, &m->gp);
        if (st == FGS_OK) st = check_gmm(m->gp);
    } else {
        st = load_pbas_params(params, &m->pp);
        if (st == FGS_OK) st = check_pbas(m->pp);
    }
    if (st != FGS_OK) {
        delete m;
        return st;
    }
    m->gc = gmm_consts(m->gp);
    m->pc.N = m->pp.N;
    m->pc.min_matches = m->pp.min_matches;
    m->pc.R_incdec = m->pp.R_incdec;
    m->pc.R_scale = m->pp.R_scale;
    m->pc.T_inc = m->pp.T_inc;
    m->pc.T_dec = m->pp.T_dec;
    m->pc.T_lower = m->pp.T_lower;
    m->pc.T_upper = m->pp.T_upper;
    for (int j = 0; j < 4; ++j) m->pc.R_lower[j] = m->pp.R_lower[j];
    m->pc.depth_max_mm = (uint32_t)m->pp.depth_max_mm;
    m->pc.key0 = (uint32_t)(m->pp.seed & 0xFFFFFFFFu);
    m->pc.key1 = (uint32_t)(m->pp.seed >> 32);
    m->pc.grad_alpha = m->pp.grad_alpha;

    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) {
        delete m;
        return fail(FGS_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    if (hip_stream) {
        m->stream = (hipStream_t)hip_stream;
        m->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete m;
            return fail(FGS_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        m->own_stream = true;
    }

    const size_t n = (size_t)m->npix;
    size_t off = 0;
    size_t o_state = 0, o_samples = 0, o_dhist = 0, o_R = 0, o_T = 0, o_S = 0, o_last = 0, o_i0 = 0,
           o_i1 = 0, o_mask = 0;
    size_t o_gs = 0, o_gsum = 0, o_lastg = 0;
    if (algo == FGS_GMM) {
        o_state = off;
        off += align256((size_t)gmm_planes(m->gp.Kc, m->gp.Kd, m->gp.var_mode) * n * 16);
    } else if (m->pp.gradient) {
        const size_t N = (size_t)m->pp.N;
        o_samples = off; off += align256(N * n * 4);
        o_gs = off;      off += align256(N * n * 4);
        o_dhist = off;   off += align256(N * n * 16);
        o_R = off;       off += align256(n * 16);
        o_T = off;       off += align256(n * 16);
        o_S = off;       off += align256(n * 16);
        o_last = off;    off += align256(n * 4);
        o_lastg = off;   off += align256(n * 4);
        o_i0 = off;      off += align256(n);
        o_i1 = off;      off += align256(n);
        o_gsum = off;    off += align256(12 * 8);
    } else {
        const size_t N = (size_t)m->pp.N;
        o_samples = off; off += align256((size_t)((N + 3) & ~3) * n * 4);  // quad planes
        o_dhist = off;   off += align256(N * n * 4);
        o_R = off;       off += align256(n * 16);
        o_T = off;       off += align256(n * 16);
        o_S = off;       off += align256(n * 8);
        o_last = off;    off += align256(n * 4);
        o_i0 = off;      off += align256(n);
        o_i1 = off;      off += align256(n);
    }
    o_mask = off;
    off += align256(n);
    m->dev_bytes = off;
    e = hipMalloc((void**)&m->dev, off);
    if (e != hipSuccess) {
        if (m->own_stream) (void)hipStreamDestroy(m->stream);
        delete m;
        return fail(FGS_ERR_OUT_OF_MEMORY, "device allocation of %zu bytes: %s", off, hipGetErrorString(e));
    }
    m->mask = m->dev + o_mask;
    if (algo == FGS_GMM) {
        m->gmm_state = reinterpret_cast<float4*>(m->dev + o_state);
        e = gmm_launch_init(m->gmm_state, m->gp.Kc, m->gp.Kd, m->npix, m->gc, m->stream);
    } else if (m->pp.gradient) {
        m->pg.samples = reinterpret_cast<uint32_t*>(m->dev + o_samples);
        m->pg.gsamples = reinterpret_cast<uint32_t*>(m->dev + o_gs);
        m->pg.D = reinterpret_cast<float4*>(m->dev + o_dhist);
        m->pg.R = reinterpret_cast<float4*>(m->dev + o_R);
        m->pg.T = reinterpret_cast<float4*>(m->dev + o_T);
        m->pg.S = reinterpret_cast<float4*>(m->dev + o_S);
        m->pg.last = reinterpret_cast<uint32_t*>(m->dev + o_last);
        m->pg.last_g = reinterpret_cast<uint32_t*>(m->dev + o_lastg);
        m->pg.fire[0] = m->dev + o_i0;
        m->pg.fire[1] = m->dev + o_i1;
        m->pg.mask = m->mask;
        m->pg.gsum = reinterpret_cast<unsigned long long*>(m->dev + o_gsum);
        e = hipMemsetAsync(m->dev, 0, off, m->stream);
        if (e == hipSuccess) e = pbas_grad_launch_init_state(m->pg, m->npix, m->pc, m->stream);
    } else {
        m->pb.samples = reinterpret_cast<uint32_t*>(m->dev + o_samples);
        m->pb.dhist = reinterpret_cast<uint32_t*>(m->dev + o_dhist);
        m->pb.R = reinterpret_cast<float4*>(m->dev + o_R);
        m->pb.T = reinterpret_cast<float4*>(m->dev + o_T);
        m->pb.S = reinterpret_cast<uint2*>(m->dev + o_S);
        m->pb.last = reinterpret_cast<uint32_t*>(m->dev + o_last);
        m->pb.fire[0] = m->dev + o_i0;
        m->pb.fire[1] = m->dev + o_i1;
        m->pb.mask = m->mask;
        // the previous value in the first padding slot (the step kernels of N >= 33 read it
        // there; smaller N keep the plane, see pbas_tile)
        m->pb.last_in_pad = (m->pp.N & 3) != 0 && m->pp.N >= 33 ? 1 : 0;
        e = hipMemsetAsync(m->dev, 0, off, m->stream);
        if (e == hipSuccess) e = pbas_launch_init_state(m->pb, m->npix, m->pc, m->stream);
    }
    if (e == hipSuccess) e = hipMemsetAsync(m->mask, 0, n, m->stream);
    if (e != hipSuccess) {
        (void)hipFree(m->dev);
        if (m->own_stream) (void)hipStreamDestroy(m->stream);
        delete m;
        return fail(FGS_ERR_DEVICE, "model initialisation: %s", hipGetErrorString(e));
    }
    m->cache_policy = FGS_CACHE_AUTO;
    if (m->device >= 0 && m->device < kMaxDevices) g_resident[m->device] += (int64_t)m->dev_bytes;
    *out = m;
    return FGS_OK;
}

fgs_status fgs_destroy(fgs_model* m) {
    if (!m) return FGS_OK;
    if (m->device >= 0 && m->device < kMaxDevices) g_resident[m->device] -= (int64_t)m->dev_bytes;
    (void)hipStreamSynchronize(m->stream);
    if (m->dev) (void)hipFree(m->dev);
    if (m->dev_in) (void)hipFree(m->dev_in);
    if (m->eval_acc) (void)hipFree(m->eval_acc);
    if (m->st_count) (void)hipFree(m->st_count);
    if (m->gt_dev) (void)hipFree(m->gt_dev);
    if (m->gt_stage) {
        (void)hipEventDestroy(m->gt_done);
        (void)hipHostFree(m->gt_stage);
    }
    if (m->host_stage) {
        (void)hipEventDestroy(m->stage_done);
        (void)hipHostFree(m->host_stage);
    }
    if (m->own_stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return FGS_OK;
}

fgs_status fgs_push_frame(fgs_model* m, const uint8_t* rgb, int64_t rgb_stride,
                          const uint16_t* depth, int64_t depth_stride, fgs_mem where) {
    if (!m) return fail(FGS_ERR_INVALID_ARG, "model is NULL");
    return fgs_push_frame_scaled(m, rgb, rgb_stride, depth, depth_stride, m->H, m->W, where);
}

fgs_status fgs_push_frame_scaled(fgs_model* m, const uint8_t* rgb, int64_t rgb_stride,
                                 const uint16_t* depth, int64_t depth_stride, int32_t depth_H,
                                 int32_t depth_W, fgs_mem where) {
    if (!m) return fail(FGS_ERR_INVALID_ARG, "model is NULL");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    if (!rgb || !depth) return fail(FGS_ERR_INVALID_ARG, "frame pointer is NULL");
    if (depth_H < 1 || depth_W < 1 || (int64_t)depth_H * depth_W > kMaxPixels)
        return fail(FGS_ERR_INVALID_ARG, "bad depth size %d x %d", depth_H, depth_W);
    if (where == FGS_MEM_HOST && (int64_t)depth_H * depth_W > (int64_t)m->npix)
        return fail(FGS_ERR_INVALID_ARG, "host depth maps may not have more pixels than the RGB frame");
    if (rgb_stride < 3 * (int64_t)m->W || depth_stride < 2 * (int64_t)depth_W || (depth_stride & 1) ||
        ((uintptr_t)depth & 1))
        return fail(FGS_ERR_INVALID_ARG, "bad stride (rgb %lld, depth %lld) for W = %d, depth W = %d",
                    (long long)rgb_stride, (long long)depth_stride, m->W, depth_W);
    const bool scaled = depth_H != m->H || depth_W != m->W;
    if (where != FGS_MEM_HOST && where != FGS_MEM_DEVICE)
        return fail(FGS_ERR_INVALID_ARG, "bad memory kind %d", (int)where);
    if (m->t >= 0xFFFFFFFFll) return fail(FGS_ERR_BAD_STATE, "frame counter exhausted");

    const uint8_t* drgb = rgb;
    const uint8_t* ddep = reinterpret_cast<const uint8_t*>(depth);
    int64_t rs = rgb_stride, ds = depth_stride;
    if (where == FGS_MEM_HOST) {
        fgs_status st = ensure_staging(m);
        if (st != FGS_OK) return st;
        if (m->stage_busy) FGS_HIP(m, hipEventSynchronize(m->stage_done));
        const size_t rgb_bytes = (size_t)m->npix * 3;
        uint8_t* hr = m->host_stage;
        uint8_t* hd = m->host_stage + align256(rgb_bytes);
        for (int y = 0; y < m->H; ++y)
            std::memcpy(hr + (size_t)y * 3 * m->W, rgb + (size_t)y * rgb_stride, (size_t)3 * m->W);
        for (int y = 0; y < depth_H; ++y)
            std::memcpy(hd + (size_t)y * 2 * depth_W, reinterpret_cast<const uint8_t*>(depth) + (size_t)y * depth_stride,
                        (size_t)2 * depth_W);
        const size_t bytes = align256(rgb_bytes) + (size_t)m->npix * 2;
        FGS_HIP(m, hipMemcpyAsync(m->dev_in, m->host_stage, bytes, hipMemcpyHostToDevice, m->stream));
        FGS_HIP(m, hipEventRecord(m->stage_done, m->stream));
        m->stage_busy = true;
        drgb = m->dev_in;
        ddep = m->dev_in + align256(rgb_bytes);
        rs = 3 * (int64_t)m->W;
        ds = 2 * (int64_t)depth_W;
    }
    const int32_t dh = scaled ? depth_H : 0, dw = scaled ? depth_W : 0;

    if (m->algo == FGS_GMM) {
        GmmStepArgs a;
        model_next_gmm(m, drgb, rs, ddep, ds, dh, dw, &a);
        FGS_HIP(m, gmm_launch_step(a, m->gp.Kc, m->gp.Kd, m->stream));
    } else if (m->pp.gradient) {
        PbasGradArgs a;
        model_next_pbas_grad(m, drgb, rs, ddep, ds, dh, dw, &a);
        FGS_HIP(m, pbas_grad_launch_step(a, m->stream));
    } else {
        PbasStepArgs a;
        model_next_pbas(m, drgb, rs, ddep, ds, dh, dw, &a);
        FGS_HIP(m, pbas_launch_step(a, m->stream));
    }
    return static_after_push(m);
}

fgs_status fgs_push_frames(fgs_model* const* models, int32_t n, const uint8_t* const* rgb,
                           const int64_t* rgb_stride, const uint16_t* const* depth,
                           const int64_t* depth_stride) {
    if (n < 1 || n > 4096) return fail(FGS_ERR_INVALID_ARG, "push_frames: n = %d outside 1..4096", n);
    if (!models || !rgb || !rgb_stride || !depth || !depth_stride)
        return fail(FGS_ERR_INVALID_ARG, "push_frames: NULL array");
    // every check first: either every model takes its frame or none does
    for (int i = 0; i < n; ++i) {
        fgs_model* m = models[i];
        if (!m) return fail(FGS_ERR_INVALID_ARG, "push_frames: model %d is NULL", i);
        if (m->poisoned) return fail(FGS_ERR_DEVICE, "push_frames: model %d is poisoned by an earlier device error", i);
        if (!rgb[i] || !depth[i]) return fail(FGS_ERR_INVALID_ARG, "push_frames: frame %d is NULL", i);
        if (rgb_stride[i] < 3 * (int64_t)m->W || depth_stride[i] < 2 * (int64_t)m->W || (depth_stride[i] & 1) ||
            ((uintptr_t)depth[i] & 1))
            return fail(FGS_ERR_INVALID_ARG, "push_frames: bad stride (rgb %lld, depth %lld) for model %d, W = %d",
                        (long long)rgb_stride[i], (long long)depth_stride[i], i, m->W);
        if (m->t >= 0xFFFFFFFFll) return fail(FGS_ERR_BAD_STATE, "push_frames: model %d frame counter exhausted", i);
        if (m->stream != models[0]->stream || m->device != models[0]->device)
            return fail(FGS_ERR_INVALID_ARG, "push_frames: model %d has another stream or device than model 0", i);
        for (int j = 0; j < i; ++j)
            if (models[j] == m) return fail(FGS_ERR_INVALID_ARG, "push_frames: model %d appears twice", i);
    }
    hipStream_t s = models[0]->stream;
    std::vector<GmmStepArgs> ga(n);
    std::vector<PbasStepArgs> pa(n);
    std::vector<PbasGradArgs> pg(n);
    std::vector<int> key(n), done(n, 0);
    for (int i = 0; i < n; ++i) {
        fgs_model* m = models[i];
        const uint8_t* d = reinterpret_cast<const uint8_t*>(depth[i]);
        if (m->algo == FGS_GMM) {
            model_next_gmm(m, rgb[i], rgb_stride[i], d, depth_stride[i], 0, 0, &ga[i]);
            key[i] = gmm_batch_key(ga[i], m->gp.Kc, m->gp.Kd);
        } else if (m->pp.gradient) {  // launched alone
            model_next_pbas_grad(m, rgb[i], rgb_stride[i], d, depth_stride[i], 0, 0, &pg[i]);
            key[i] = -2;
        } else {
            model_next_pbas(m, rgb[i], rgb_stride[i], d, depth_stride[i], 0, 0, &pa[i]);
            key[i] = pbas_batch_key(pa[i]);
        }
    }
    // models of one kind and key share a launch (up to kBatchMax each); fill frames go alone.
    // Every frame counter has advanced: a failed launch poisons its models and every model
    // whose launch had not been issued yet.
    auto fail_group = [&](const std::vector<int>& idx, hipError_t e) {
        for (int k : idx) models[k]->poisoned = true;
        for (int k = 0; k < n; ++k)
            if (!done[k]) models[k]->poisoned = true;
        return device_fail(models[idx[0]], e, "push_frames");
    };
    for (int i = 0; i < n; ++i) {
        if (done[i]) continue;
        fgs_model* m = models[i];
        std::vector<int> idx;
        for (int j = i; j < n && (int)idx.size() < kBatchMax; ++j)
            if (!done[j] && models[j]->algo == m->algo && key[j] == key[i] &&
                (m->algo == FGS_PBAS || (models[j]->gp.Kc == m->gp.Kc && models[j]->gp.Kd == m->gp.Kd)) &&
                (key[i] >= 0 || j == i))
                idx.push_back(j);
        for (int k : idx) done[k] = 1;
        hipError_t e;
        if (m->algo == FGS_GMM) {
            GmmStepArgs b[kBatchMax];
            for (size_t k = 0; k < idx.size(); ++k) b[k] = ga[idx[k]];
            e = gmm_launch_step_batch(b, (int)idx.size(), m->gp.Kc, m->gp.Kd, s);
        } else if (key[i] == -2) {
            e = pbas_grad_launch_step(pg[i], s);
        } else if (key[i] < 0) {
            e = pbas_launch_step(pa[i], s);
        } else {
            PbasStepArgs b[kBatchMax];
            for (size_t k = 0; k < idx.size(); ++k) b[k] = pa[idx[k]];
            e = pbas_launch_step_batch(b, (int)idx.size(), s);
        }
        if (e != hipSuccess) return fail_group(idx, e);
    }
    for (int i = 0; i < n; ++i) {
        const fgs_status st = static_after_push(models[i]);
        if (st != FGS_OK) return st;
    }
    return FGS_OK;
}

fgs_status fgs_get_mask(fgs_model* m, uint8_t* mask, int64_t stride, fgs_mem where) {
    if (!m || !mask) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    if (stride < m->W) return fail(FGS_ERR_INVALID_ARG, "mask stride %lld < W", (long long)stride);
    if (m->t == 0) return fail(FGS_ERR_BAD_STATE, "no frame has been pushed");
    if (where == FGS_MEM_HOST) {
        FGS_HIP(m, hipMemcpy2DAsync(mask, (size_t)stride, m->mask, (size_t)m->W, (size_t)m->W,
                                    (size_t)m->H, hipMemcpyDeviceToHost, m->stream));
        FGS_HIP(m, hipStreamSynchronize(m->stream));
    } else if (where == FGS_MEM_DEVICE) {
        FGS_HIP(m, hipMemcpy2DAsync(mask, (size_t)stride, m->mask, (size_t)m->W, (size_t)m->W,
                                    (size_t)m->H, hipMemcpyDeviceToDevice, m->stream));
    } else {
        return fail(FGS_ERR_INVALID_ARG, "bad memory kind %d", (int)where);
    }
    return FGS_OK;
}

fgs_status fgs_static_enable(fgs_model* m, int32_t M) {
    if (!m) return fail(FGS_ERR_INVALID_ARG, "model is NULL");
    if (M < 0 || M > 65535) return fail(FGS_ERR_INVALID_ARG, "M = %d outside 0..65535", M);
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    if (M == 0) {
        if (m->st_count) {
            FGS_HIP(m, hipStreamSynchronize(m->stream));
            (void)hipFree(m->st_count);
        }
        m->st_count = nullptr;
        m->st_mask = nullptr;
        m->st_M = 0;
        m->st_frames = 0;
        return FGS_OK;
    }
    const size_t n = (size_t)m->npix;
    if (!m->st_count) {
        uint8_t* p = nullptr;
        hipError_t e = hipMalloc((void**)&p, align256(n * 2) + align256(n));
        if (e != hipSuccess) return fail(FGS_ERR_OUT_OF_MEMORY, "static-object planes: %s", hipGetErrorString(e));
        m->st_count = reinterpret_cast<uint16_t*>(p);
        m->st_mask = p + align256(n * 2);
    }
    FGS_HIP(m, static_launch_clear(m->st_count, m->st_mask, m->npix, m->stream));
    m->st_M = M;
    m->st_frames = 0;
    return FGS_OK;
}

fgs_status fgs_static_mask(fgs_model* m, uint8_t* out, int64_t stride, fgs_mem where) {
    if (!m || !out) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    if (stride < m->W) return fail(FGS_ERR_INVALID_ARG, "mask stride %lld < W", (long long)stride);
    if (where != FGS_MEM_HOST && where != FGS_MEM_DEVICE)
        return fail(FGS_ERR_INVALID_ARG, "bad memory kind %d", (int)where);
    if (m->st_M <= 0) return fail(FGS_ERR_BAD_STATE, "static-object detection is not enabled");
    if (m->st_frames == 0) return fail(FGS_ERR_BAD_STATE, "no frame has been counted since it was enabled");
    FGS_HIP(m, hipMemcpy2DAsync(out, (size_t)stride, m->st_mask, (size_t)m->W, (size_t)m->W, (size_t)m->H,
                                where == FGS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                m->stream));
    if (where == FGS_MEM_HOST) FGS_HIP(m, hipStreamSynchronize(m->stream));
    return FGS_OK;
}

fgs_status fgs_mask_device_ptr(fgs_model* m, const uint8_t** out) {
    if (!m || !out) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    *out = m->mask;
    return FGS_OK;
}

namespace {

fgs_status ensure_eval(fgs_model* m) {
    if (m->eval_acc) return FGS_OK;
    hipError_t e = hipMalloc((void**)&m->eval_acc, 4 * kEvalSlots * sizeof(unsigned long long));
    if (e != hipSuccess) {
        m->eval_acc = nullptr;
        return fail(FGS_ERR_OUT_OF_MEMORY, "evaluation counters: %s", hipGetErrorString(e));
    }
    FGS_HIP(m, eval_launch_zero(m->eval_acc, m->stream));
    return FGS_OK;
}

fgs_status ensure_gt_staging(fgs_model* m) {
    if (m->gt_stage) return FGS_OK;
    hipError_t e = hipHostMalloc((void**)&m->gt_stage, (size_t)m->npix, hipHostMallocDefault);
    if (e != hipSuccess) {
        m->gt_stage = nullptr;
        return fail(FGS_ERR_OUT_OF_MEMORY, "pinned ground-truth staging: %s", hipGetErrorString(e));
    }
    e = hipMalloc((void**)&m->gt_dev, (size_t)m->npix);
    if (e != hipSuccess) {
        (void)hipHostFree(m->gt_stage);
        m->gt_stage = nullptr;
        m->gt_dev = nullptr;
        return fail(FGS_ERR_OUT_OF_MEMORY, "device ground-truth staging: %s", hipGetErrorString(e));
    }
    FGS_HIP(m, hipEventCreateWithFlags(&m->gt_done, hipEventDisableTiming));
    m->gt_busy = false;
    return FGS_OK;
}

}  // namespace

fgs_status fgs_eval_accumulate(fgs_model* m, const uint8_t* gt, int64_t gt_stride, fgs_mem where) {
    if (!m || !gt) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    if (gt_stride < m->W) return fail(FGS_ERR_INVALID_ARG, "ground-truth stride %lld < W", (long long)gt_stride);
    if (where != FGS_MEM_HOST && where != FGS_MEM_DEVICE)
        return fail(FGS_ERR_INVALID_ARG, "bad memory kind %d", (int)where);
    if (m->t == 0) return fail(FGS_ERR_BAD_STATE, "no frame has been pushed");
    fgs_status st = ensure_eval(m);
    if (st != FGS_OK) return st;
    const uint8_t* dgt = gt;
    int64_t gs = gt_stride;
    if (where == FGS_MEM_HOST) {
        st = ensure_gt_staging(m);
        if (st != FGS_OK) return st;
        if (m->gt_busy) FGS_HIP(m, hipEventSynchronize(m->gt_done));
        for (int y = 0; y < m->H; ++y)
            std::memcpy(m->gt_stage + (size_t)y * m->W, gt + (size_t)y * gt_stride, (size_t)m->W);
        FGS_HIP(m, hipMemcpyAsync(m->gt_dev, m->gt_stage, (size_t)m->npix, hipMemcpyHostToDevice, m->stream));
        FGS_HIP(m, hipEventRecord(m->gt_done, m->stream));
        m->gt_busy = true;
        dgt = m->gt_dev;
        gs = m->W;
    }
    FGS_HIP(m, eval_launch_count(m->mask, dgt, gs, m->H, m->W, m->eval_acc, m->stream));
    return FGS_OK;
}

fgs_status fgs_eval_read(fgs_model* m, uint64_t counts[4], int32_t reset) {
    if (!m || !counts) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    if (!m->eval_acc) {
        for (int i = 0; i < 4; ++i) counts[i] = 0;
        return FGS_OK;
    }
    unsigned long long v[4 * kEvalSlots];
    FGS_HIP(m, hipMemcpyAsync(v, m->eval_acc, sizeof v, hipMemcpyDeviceToHost, m->stream));
    FGS_HIP(m, hipStreamSynchronize(m->stream));
    for (int i = 0; i < 4; ++i) {
        uint64_t c = 0;
        for (int k = 0; k < kEvalSlots; ++k) c += (uint64_t)v[i * kEvalSlots + k];
        counts[i] = c;
    }
    if (reset) FGS_HIP(m, eval_launch_zero(m->eval_acc, m->stream));
    return FGS_OK;
}

fgs_status fgs_state_size(const fgs_model* m, size_t* bytes) {
    if (!m || !bytes) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    *bytes = kHeaderBytes + payload_bytes(m);
    return FGS_OK;
}

namespace {

// Device staging of fgs_copy_state_noalloc: a file-scope array that each GPU the library
// runs on holds from its first use until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in for the symbol):
// it uses the device address hipGetSymbolAddress returns, looked up once per device with
// that device current and kept in g_noalloc_ptr.
std::atomic<uint8_t*> g_noalloc_ptr[kMaxDevices];

fgs_status noalloc_staging(int device, uint8_t** out) {
    if (device < 0 || device >= kMaxDevices) return fail(FGS_ERR_DEVICE, "device %d out of range", device);
    uint8_t* p = g_noalloc_ptr[device].load(std::memory_order_acquire);
    if (!p) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void* addr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !addr)
            return fail(FGS_ERR_DEVICE, "staging buffer address on device %d: %s", device,
                        hipGetErrorString(e != hipSuccess ? e : hipErrorInvalidSymbol));
        p = reinterpret_cast<uint8_t*>(addr);
        g_noalloc_ptr[device].store(p, std::memory_order_release);  // the same address if two threads race here
    }
    *out = p;
    return FGS_OK;
}

// fgs_copy_state with a host destination staged through `staging` (nullptr: a buffer
// allocated for this call and freed after it).
fgs_status copy_state_impl(fgs_model* m, void* dst, size_t bytes, fgs_mem where, uint8_t* staging) {

    if (!m || !dst) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    const size_t payload = payload_bytes(m);
    if (bytes != kHeaderBytes + payload)
        return fail(FGS_ERR_INVALID_ARG, "state buffer is %zu bytes, need %zu", bytes, kHeaderBytes + payload);
    if (where != FGS_MEM_HOST && where != FGS_MEM_DEVICE)
        return fail(FGS_ERR_INVALID_ARG, "bad memory kind %d", (int)where);
    if (where == FGS_MEM_DEVICE && ((uintptr_t)dst & 3))
        return fail(FGS_ERR_INVALID_ARG, "device state buffer must be 4-byte aligned");
    fgs_status st = flush_pending(m);
    if (st != FGS_OK) return st;

    StateHeader h;
    std::memset(&h, 0, sizeof h);
    h.magic = kStateMagic;
    h.version = kStateVersion;
    h.algo = (uint32_t)m->algo;
    h.H = m->H;
    h.W = m->W;
    h.A = m->algo == FGS_GMM ? m->gp.Kc : m->pp.N;
    h.B = m->algo == FGS_GMM ? m->gp.Kd : 0;
    h.flags = m->algo == FGS_GMM ? m->gp.var_mode : (m->pp.gradient ? 2 : 0);
    h.frames = m->t;
    h.seed = m->algo == FGS_PBAS ? m->pp.seed : 0;

    uint8_t* tmp = nullptr;
    uint8_t* target = reinterpret_cast<uint8_t*>(dst) + kHeaderBytes;
    if (where == FGS_MEM_HOST) {
        if (staging) {
            target = staging;
        } else {
            FGS_HIP(m, hipMalloc((void**)&tmp, payload));
            target = tmp;
        }
    }
    hipError_t e = m->algo == FGS_GMM
                       ? gmm_launch_export(m->gmm_state, reinterpret_cast<float*>(target), m->gp.Kc,
                                           m->gp.Kd, m->gp.var_mode, m->npix, m->stream)
                       : m->pp.gradient ? pbas_grad_launch_export(m->pg, m->npix, m->pp.N, m->t, target, m->stream)
                                        : pbas_launch_export(m->pb, m->npix, m->pp.N, target, m->stream);
    if (e == hipSuccess) {
        if (where == FGS_MEM_HOST) {
            std::memcpy(dst, &h, sizeof h);
            e = hipMemcpyAsync(reinterpret_cast<uint8_t*>(dst) + kHeaderBytes, target, payload,
                               hipMemcpyDeviceToHost, m->stream);
        } else {
            e = hipMemcpyAsync(dst, &h, sizeof h, hipMemcpyHostToDevice, m->stream);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return device_fail(m, e, "copy_state");
    return FGS_OK;
}

}  // namespace

fgs_status fgs_copy_state(fgs_model* m, void* dst, size_t bytes, fgs_mem where) {
    return copy_state_impl(m, dst, bytes, where, nullptr);
}

fgs_status fgs_copy_state_noalloc(fgs_model* m, void* dst, size_t bytes, fgs_mem where) {
    if (!m || !dst) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    uint8_t* staging = nullptr;
    if (where == FGS_MEM_HOST) {
        const size_t payload = payload_bytes(m);
        if (bytes != kHeaderBytes + payload)
            return fail(FGS_ERR_INVALID_ARG, "state buffer is %zu bytes, need %zu", bytes, kHeaderBytes + payload);
        if (payload > kNoallocBytes)
            return fail(FGS_ERR_UNSUPPORTED,
                        "state payload of %zu bytes exceeds the %zu-byte staging buffer of the "
                        "allocation-free copy (use fgs_copy_state or a device destination)",
                        payload, kNoallocBytes);
        fgs_status st = noalloc_staging(m->device, &staging);
        if (st != FGS_OK) return st;
    }
    return copy_state_impl(m, dst, bytes, where, staging);
}

fgs_status fgs_set_state(fgs_model* m, const void* src, size_t bytes, fgs_mem where) {
    if (!m || !src) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    const size_t payload = payload_bytes(m);
    if (bytes != kHeaderBytes + payload)
        return fail(FGS_ERR_INVALID_ARG, "state blob is %zu bytes, need %zu", bytes, kHeaderBytes + payload);
    if (where != FGS_MEM_HOST && where != FGS_MEM_DEVICE)
        return fail(FGS_ERR_INVALID_ARG, "bad memory kind %d", (int)where);
    if (where == FGS_MEM_DEVICE && ((uintptr_t)src & 3))
        return fail(FGS_ERR_INVALID_ARG, "device state blob must be 4-byte aligned");
    StateHeader h;
    if (where == FGS_MEM_HOST) {
        std::memcpy(&h, src, sizeof h);
    } else {
        FGS_HIP(m, hipMemcpyAsync(&h, src, sizeof h, hipMemcpyDeviceToHost, m->stream));
        FGS_HIP(m, hipStreamSynchronize(m->stream));
    }
    const int A = m->algo == FGS_GMM ? m->gp.Kc : m->pp.N;
    const int B = m->algo == FGS_GMM ? m->gp.Kd : 0;
    if (h.magic != kStateMagic || h.version != kStateVersion || h.algo != (uint32_t)m->algo ||
        h.H != m->H || h.W != m->W || h.A != A || h.B != B || h.frames < 0 || h.frames >= 0xFFFFFFFFll ||
        h.flags != (m->algo == FGS_GMM ? m->gp.var_mode : (m->pp.gradient ? 2 : 0)))
        return fail(FGS_ERR_INVALID_ARG, "state header does not match this model");
    if (m->algo == FGS_PBAS && h.seed != m->pp.seed)
        return fail(FGS_ERR_INVALID_ARG, "state was taken with another PBAS seed");

    uint8_t* tmp = nullptr;
    const uint8_t* srcp = reinterpret_cast<const uint8_t*>(src) + kHeaderBytes;
    hipError_t e = hipSuccess;
    if (where == FGS_MEM_HOST) {
        FGS_HIP(m, hipMalloc((void**)&tmp, payload));
        e = hipMemcpyAsync(tmp, srcp, payload, hipMemcpyHostToDevice, m->stream);
        srcp = tmp;
    }
    if (e == hipSuccess)
        e = m->algo == FGS_GMM ? gmm_launch_import(m->gmm_state, reinterpret_cast<const float*>(srcp),
                                                   m->gp.Kc, m->gp.Kd, m->gp.var_mode, m->npix, m->stream)
                               : m->pp.gradient
                                     ? pbas_grad_launch_import(m->pg, m->npix, m->pp.N, h.frames, srcp, m->stream)
                                     : pbas_launch_import(m->pb, m->npix, m->pp.N, srcp, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (tmp) (void)hipFree(tmp);
    if (e != hipSuccess) return device_fail(m, e, "set_state");
    m->t = h.frames;
    m->pending = false;
    if (m->st_M > 0) {  // the detector's runs restart with the new state
        FGS_HIP(m, static_launch_clear(m->st_count, m->st_mask, m->npix, m->stream));
        m->st_frames = 0;
    }
    return FGS_OK;
}

fgs_status fgs_get_state(fgs_model* m, fgs_state_field* fields, int32_t capacity, int32_t* count) {
    if (!m || !count) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (m->poisoned) return fail(FGS_ERR_DEVICE, "model is poisoned by an earlier device error");
    std::vector<fgs_state_field> f;
    auto add = [&](const char* name, int index, int sub, int dtype, int bytes, const uint8_t* base,
                   int64_t stride) {
        f.push_back(fgs_state_field{name, index, sub, dtype, bytes, base, stride});
    };
    const int64_t n = m->npix;
    if (m->algo == FGS_GMM) {
        const int Kc = m->gp.Kc, Kd = m->gp.Kd, var = m->gp.var_mode;
        const uint8_t* st = reinterpret_cast<const uint8_t*>(m->gmm_state);
        auto core = [&](int k, int lane) { return st + (int64_t)k * n * 16 + 4 * lane; };
        auto extra = [&](int i) { return st + (int64_t)(Kc + i / 4) * n * 16 + 4 * (i % 4); };
        for (int k = 0; k < Kc; ++k) add("w_c", k, 0, FGS_DTYPE_F32, 4, extra(gmm_x_wc(Kc, Kd, k)), 16);
        for (int k = 0; k < Kc; ++k)
            for (int c = 0; c < 3; ++c) add("mu_c", k, c, FGS_DTYPE_F32, 4, core(k, c), 16);
        for (int k = 0; k < Kc; ++k) {
            add("v_c", k, 0, FGS_DTYPE_F32, 4, core(k, 3), 16);
            if (var) {
                add("v_c", k, 1, FGS_DTYPE_F32, 4, extra(gmm_x_vg(Kc, Kd, k)), 16);
                add("v_c", k, 2, FGS_DTYPE_F32, 4, extra(gmm_x_vb(Kc, Kd, k)), 16);
            }
        }
        for (int k = 0; k < Kd; ++k) add("w_d", k, 0, FGS_DTYPE_F32, 4, extra(gmm_x_wd(Kc, Kd, k)), 16);
        for (int k = 0; k < Kd; ++k) add("mu_d", k, 0, FGS_DTYPE_F32, 4, extra(gmm_x_mud(Kc, Kd, k)), 16);
        for (int k = 0; k < Kd; ++k) add("v_d", k, 0, FGS_DTYPE_F32, 4, extra(gmm_x_vd(Kc, Kd, k)), 16);
    } else if (m->pp.gradient) {
        const int N = m->pp.N;
        const uint8_t* smp = reinterpret_cast<const uint8_t*>(m->pg.samples);
        const uint8_t* gsm = reinterpret_cast<const uint8_t*>(m->pg.gsamples);
        const uint8_t* dh = reinterpret_cast<const uint8_t*>(m->pg.D);
        for (int k = 0; k < N; ++k) add("samples", k, 0, FGS_DTYPE_U32, 4, smp + (int64_t)k * n * 4, 4);
        for (int k = 0; k < N; ++k) add("gsamples", k, 0, FGS_DTYPE_U32, 4, gsm + (int64_t)k * n * 4, 4);
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < 4; ++j) add("dhist", k, j, FGS_DTYPE_F32, 4, dh + (int64_t)k * n * 16 + 4 * j, 16);
        for (int j = 0; j < 4; ++j)
            add("R", j, 0, FGS_DTYPE_F32, 4, reinterpret_cast<const uint8_t*>(m->pg.R) + 4 * j, 16);
        for (int j = 0; j < 4; ++j)
            add("T", j, 0, FGS_DTYPE_F32, 4, reinterpret_cast<const uint8_t*>(m->pg.T) + 4 * j, 16);
        for (int j = 0; j < 4; ++j)
            add("S", j, 0, FGS_DTYPE_F32, 4, reinterpret_cast<const uint8_t*>(m->pg.S) + 4 * j, 16);
    } else {
        const int N = m->pp.N;
        const uint8_t* smp = reinterpret_cast<const uint8_t*>(m->pb.samples);
        const uint8_t* dh = reinterpret_cast<const uint8_t*>(m->pb.dhist);
        for (int k = 0; k < N; ++k)  // quad planes: slot k is word k & 3 of quad (k >> 2)
            add("samples", k, 0, FGS_DTYPE_U32, 4, smp + (int64_t)(k >> 2) * n * 16 + 4 * (k & 3), 16);
        for (int k = 0; k < N; ++k) add("dhist", k, 0, FGS_DTYPE_U32, 4, dh + (int64_t)k * n * 4, 4);
        for (int j = 0; j < 4; ++j)
            add("R", j, 0, FGS_DTYPE_F32, 4, reinterpret_cast<const uint8_t*>(m->pb.R) + 4 * j, 16);
        for (int j = 0; j < 4; ++j)
            add("T", j, 0, FGS_DTYPE_F32, 4, reinterpret_cast<const uint8_t*>(m->pb.T) + 4 * j, 16);
        for (int j = 0; j < 4; ++j)
            add("S", j, 0, FGS_DTYPE_U16, 2, reinterpret_cast<const uint8_t*>(m->pb.S) + 2 * j, 8);
    }
    const int32_t need = (int32_t)f.size();
    *count = need;
    if (!fields) return FGS_OK;
    if (capacity < need) return fail(FGS_ERR_INVALID_ARG, "capacity %d < %d fields", capacity, need);
    fgs_status s = flush_pending(m);
    if (s != FGS_OK) return s;
    std::copy(f.begin(), f.end(), fields);
    return FGS_OK;
}

fgs_status fgs_frame_index(const fgs_model* m, int64_t* t) {
    if (!m || !t) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    *t = m->t;
    return FGS_OK;
}

fgs_status fgs_sync(fgs_model* m) {
    if (!m) return fail(FGS_ERR_INVALID_ARG, "model is NULL");
    FGS_HIP(m, hipStreamSynchronize(m->stream));
    return FGS_OK;
}

fgs_status fgs_stream(const fgs_model* m, void** hip_stream) {
    if (!m || !hip_stream) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    *hip_stream = (void*)m->stream;
    return FGS_OK;
}

fgs_status fgs_device_bytes(const fgs_model* m, size_t* bytes) {
    if (!m || !bytes) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    size_t b = m->dev_bytes;
    if (m->dev_in) b += align256((size_t)m->npix * 3) + align256((size_t)m->npix * 2);
    if (m->st_count) b += align256((size_t)m->npix * 2) + align256((size_t)m->npix);
    *bytes = b;
    return FGS_OK;
}

fgs_status fgs_set_cache_policy(fgs_model* m, int32_t policy) {
    if (!m) return fail(FGS_ERR_INVALID_ARG, "model is NULL");
    if (policy != FGS_CACHE_AUTO && policy != FGS_CACHE_KEEP && policy != FGS_CACHE_STREAM)
        return fail(FGS_ERR_INVALID_ARG, "unknown cache policy %d", policy);
    m->cache_policy = policy;
    return FGS_OK;
}

// ------------------------------------------------------------ GMM adjoint
}  // extern "C"

struct fgs_gmm_window {
    int32_t T, H, W, npix, K, E, nseg;
    GmmConsts c;
    hipStream_t stream;
    bool own_stream;
    uint8_t* dev;
    uint64_t* rec;
    float* ckpt;
    float* scratch;
    double* partial;
    bool have_forward;
};

extern "C" {

fgs_status fgs_gmm_window_create(int32_t T, int32_t H, int32_t W, const fgs_gmm_params* params,
                                 int32_t checkpoint_every, void* hip_stream, fgs_gmm_window** out) {
    if (!out) return fail(FGS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    fgs_gmm_params p;
    fgs_status st = load_gmm_params(params, &p);
    if (st == FGS_OK) st = check_gmm(p);
    if (st != FGS_OK) return st;
    if (p.rho_mode != 0 || p.decision != 0 || p.var_mode != 0)
        return fail(FGS_ERR_UNSUPPORTED, "the adjoint is derived for rho = alpha, the Z score and one "
                                         "variance per Gaussian (rho_mode, decision, var_mode 0)");
    if (p.Kc != p.Kd || !gmm_window_supported(p.Kc))
        return fail(FGS_ERR_UNSUPPORTED, "the adjoint supports Kc = Kd in 1..5, not (%d, %d)", p.Kc, p.Kd);
    if (T < 1 || H < 1 || W < 1 || (int64_t)H * W > kMaxPixels || checkpoint_every < 1)
        return fail(FGS_ERR_INVALID_ARG, "bad window T=%d H=%d W=%d E=%d", T, H, W, checkpoint_every);
    fgs_gmm_window* w = new (std::nothrow) fgs_gmm_window();
    if (!w) return fail(FGS_ERR_OUT_OF_MEMORY, "host allocation");
    w->T = T;
    w->H = H;
    w->W = W;
    w->npix = H * W;
    w->K = p.Kc;
    w->E = checkpoint_every < T ? checkpoint_every : T;
    w->nseg = (T + w->E - 1) / w->E;
    w->c = gmm_consts(p);
    const size_t n = (size_t)w->npix, F = 6 * (size_t)w->K;
    const size_t o_rec = 0;
    const size_t o_ckpt = o_rec + align256((size_t)T * n * 8);
    const size_t o_scr = o_ckpt + align256((size_t)w->nseg * F * n * 4);
    const size_t o_par = o_scr + align256((size_t)w->E * F * n * 4);
    const size_t total = o_par + align256((size_t)gmm_window_blocks(w->npix) * 3 * 8);
    hipError_t e = hipSuccess;
    if (hip_stream) {
        w->stream = (hipStream_t)hip_stream;
    } else {
        e = hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking);
        w->own_stream = e == hipSuccess;
    }
    if (e == hipSuccess) e = hipMalloc((void**)&w->dev, total);
    if (e != hipSuccess) {
        if (w->own_stream) (void)hipStreamDestroy(w->stream);
        delete w;
        return fail(FGS_ERR_OUT_OF_MEMORY, "window allocation of %zu bytes: %s", total, hipGetErrorString(e));
    }
    w->rec = reinterpret_cast<uint64_t*>(w->dev + o_rec);
    w->ckpt = reinterpret_cast<float*>(w->dev + o_ckpt);
    w->scratch = reinterpret_cast<float*>(w->dev + o_scr);
    w->partial = reinterpret_cast<double*>(w->dev + o_par);
    *out = w;
    return FGS_OK;
}

static GmmWindowArgs window_args(fgs_gmm_window* w, const float* theta, const uint8_t* rgb,
                                 const uint16_t* depth) {
    GmmWindowArgs a;
    std::memset(&a, 0, sizeof a);
    a.T = w->T;
    a.H = w->H;
    a.W = w->W;
    a.npix = w->npix;
    a.E = w->E;
    a.nseg = w->nseg;
    a.c = w->c;
    a.theta = theta;
    a.rgb = rgb;
    a.depth = depth;
    a.rec = w->rec;
    a.ckpt = w->ckpt;
    a.scratch = w->scratch;
    a.partial = w->partial;
    return a;
}

fgs_status fgs_gmm_window_forward(fgs_gmm_window* w, const float* theta, const uint8_t* rgb,
                                  const uint16_t* depth, float* Z, uint8_t* has_term) {
    if (!w || !theta || !rgb || !depth || !Z || !has_term) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (((uintptr_t)depth & 1) || ((uintptr_t)Z & 3) || ((uintptr_t)theta & 3))
        return fail(FGS_ERR_INVALID_ARG, "misaligned device buffer");
    GmmWindowArgs a = window_args(w, theta, rgb, depth);
    a.Z = Z;
    a.has = has_term;
    hipError_t e = gmm_window_launch_forward(a, w->K, w->stream);
    if (e != hipSuccess) return fail(FGS_ERR_DEVICE, "window forward: %s", hipGetErrorString(e));
    w->have_forward = true;
    return FGS_OK;
}

fgs_status fgs_gmm_window_backward(fgs_gmm_window* w, const float* theta, const uint8_t* rgb,
                                   const uint16_t* depth, const float* dZ, double* dtheta) {
    if (!w || !theta || !rgb || !depth || !dZ || !dtheta) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (!w->have_forward) return fail(FGS_ERR_BAD_STATE, "backward before forward");
    if (((uintptr_t)depth & 1) || ((uintptr_t)dZ & 3) || ((uintptr_t)dtheta & 7) || ((uintptr_t)theta & 3))
        return fail(FGS_ERR_INVALID_ARG, "misaligned device buffer");
    GmmWindowArgs a = window_args(w, theta, rgb, depth);
    a.dZ = dZ;
    a.dtheta = dtheta;
    hipError_t e = gmm_window_launch_backward(a, w->K, w->stream);
    if (e != hipSuccess) return fail(FGS_ERR_DEVICE, "window backward: %s", hipGetErrorString(e));
    return FGS_OK;
}

fgs_status fgs_gmm_window_records(fgs_gmm_window* w, uint64_t* out, fgs_mem where) {
    if (!w || !out) return fail(FGS_ERR_INVALID_ARG, "NULL argument");
    if (!w->have_forward) return fail(FGS_ERR_BAD_STATE, "no forward has run");
    const size_t bytes = (size_t)w->T * w->npix * 8;
    hipError_t e = hipMemcpyAsync(out, w->rec, bytes,
                                  where == FGS_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                  w->stream);
    if (e == hipSuccess && where == FGS_MEM_HOST) e = hipStreamSynchronize(w->stream);
    if (e != hipSuccess) return fail(FGS_ERR_DEVICE, "records copy: %s", hipGetErrorString(e));
    return FGS_OK;
}

fgs_status fgs_gmm_window_destroy(fgs_gmm_window* w) {
    if (!w) return FGS_OK;
    (void)hipStreamSynchronize(w->stream);
    (void)hipFree(w->dev);
    if (w->own_stream) (void)hipStreamDestroy(w->stream);
    delete w;
    return FGS_OK;
}

fgs_status fgs_mask_median(const uint8_t* src, int64_t src_stride, uint8_t* dst, int64_t dst_stride,
                           int32_t H, int32_t W, int32_t radius, void* hip_stream) {
    constexpr int32_t kMaxSide = 1 << 30;
    constexpr int64_t kMaxStride = (int64_t)1 << 32;
    if (H < 0 || W < 0 || H > kMaxSide || W > kMaxSide || (int64_t)H * W > ((int64_t)1 << 34))
        return fail(FGS_ERR_INVALID_ARG, "median: image %d x %d outside 0..2^30 per side, 2^34 pixels", H, W);
    if (radius < 0 || radius > kMedRadiusMax)
        return fail(FGS_ERR_INVALID_ARG, "median: radius %d outside 0..%d", radius, kMedRadiusMax);
    if (H == 0 || W == 0) return FGS_OK;
    if (!src || !dst) return fail(FGS_ERR_INVALID_ARG, "median: NULL buffer");
    if (src_stride < W || dst_stride < W || src_stride > kMaxStride || dst_stride > kMaxStride)
        return fail(FGS_ERR_INVALID_ARG, "median: strides %lld, %lld outside W..2^32", (long long)src_stride,
                    (long long)dst_stride);
    const uintptr_t s0 = (uintptr_t)src, s1 = s0 + (uintptr_t)((int64_t)(H - 1) * src_stride + W);
    const uintptr_t d0 = (uintptr_t)dst, d1 = d0 + (uintptr_t)((int64_t)(H - 1) * dst_stride + W);
    if (s0 < d1 && d0 < s1) return fail(FGS_ERR_INVALID_ARG, "median: source and destination overlap");
    hipError_t e = post_launch_median(src, src_stride, dst, dst_stride, H, W, radius, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(FGS_ERR_DEVICE, "median kernel: %s", hipGetErrorString(e));
    return FGS_OK;
}

fgs_status fgs_philox4x32_10(uint64_t seed, const uint32_t* ctr, uint32_t* out, int64_t n,
                             void* hip_stream) {
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(FGS_ERR_INVALID_ARG, "bad philox arguments");
    if (((uintptr_t)ctr & 15) || ((uintptr_t)out & 15))
        return fail(FGS_ERR_INVALID_ARG, "philox buffers must be 16-byte aligned");
    hipError_t e = diag_launch_philox(seed, ctr, out, n, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(FGS_ERR_DEVICE, "philox kernel: %s", hipGetErrorString(e));
    return FGS_OK;
}

fgs_status fgs_copy_probe(const void* src, void* dst, size_t bytes, void* hip_stream) {
    if (!src || !dst || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return fail(FGS_ERR_INVALID_ARG, "copy probe needs 16-byte aligned buffers and size");
    hipError_t e = diag_launch_copy(src, dst, bytes, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(FGS_ERR_DEVICE, "copy kernel: %s", hipGetErrorString(e));
    return FGS_OK;
}

fgs_status fgs_mix_probe(void* planes, int64_t npix, int32_t mode, void* hip_stream) {
    if (!planes || npix <= 0 || ((uintptr_t)planes & 15))
        return fail(FGS_ERR_INVALID_ARG, "mix probe needs a 16-byte aligned buffer and npix > 0");
    if (mode < 0 || mode > 4) return fail(FGS_ERR_INVALID_ARG, "mix probe mode %d outside 0..4", (int)mode);
    hipError_t e = diag_launch_mix(planes, npix, mode, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(FGS_ERR_DEVICE, "mix probe kernel: %s", hipGetErrorString(e));
    return FGS_OK;
}

}  // extern "C"
