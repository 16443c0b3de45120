"""ctypes binding of libfgs (include/fgs.h): same names, argument marshalling only.

Every step of the classify-and-update path runs in the library's HIP kernels.
There is no fallback: if libfgs.so is missing or fails to load, every call
raises.  PyTorch is used only for device memory and streams (``Model`` accepts
torch tensors and ``torch.cuda.Stream``s).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfgs.so")

FGS_OK = 0
FGS_ERR_INVALID_ARG = 1
FGS_ERR_OUT_OF_MEMORY = 2
FGS_ERR_DEVICE = 3
FGS_ERR_BAD_STATE = 4
FGS_ERR_BUSY = 5
FGS_ERR_UNSUPPORTED = 6

FGS_GMM = 1
FGS_PBAS = 2
FGS_MEM_HOST = 0
FGS_MEM_DEVICE = 1
FGS_CACHE_AUTO = 0
FGS_CACHE_KEEP = 1
FGS_CACHE_STREAM = 2
STATE_HEADER_BYTES = 64
ABI_VERSION = 6          # FGS_ABI_VERSION of include/fgs.h this binding is written against


class FgsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fgs status {status}: {msg}")
        self.status = status


class fgs_gmm_params(ctypes.Structure):
    _fields_ = [("struct_size", c_uint32), ("Kc", c_int32), ("Kd", c_int32),
                ("alpha", ctypes.c_float), ("lambda_", ctypes.c_float), ("T_bg", ctypes.c_float),
                ("w_init", ctypes.c_float), ("v_init_c", ctypes.c_float), ("v_min_c", ctypes.c_float),
                ("v_init_d", ctypes.c_float), ("v_min_d", ctypes.c_float), ("w_depth", ctypes.c_float),
                ("depth_max_mm", c_int32), ("rho_mode", c_int32), ("decision", c_int32),
                ("density_scale", ctypes.c_float), ("density_threshold", ctypes.c_float),
                ("var_mode", c_int32)]


class fgs_pbas_params(ctypes.Structure):
    _fields_ = [("struct_size", c_uint32), ("N", c_int32), ("min_matches", c_int32),
                ("R_incdec", ctypes.c_float), ("R_scale", ctypes.c_float),
                ("T_inc", ctypes.c_float), ("T_dec", ctypes.c_float),
                ("T_lower", ctypes.c_float), ("T_upper", ctypes.c_float),
                ("R_lower", ctypes.c_float * 4), ("depth_max_mm", c_int32), ("gradient", c_int32),
                ("seed", c_uint64), ("grad_alpha", ctypes.c_float), ("reserved1", c_int32)]


class fgs_server_stats(ctypes.Structure):
    _fields_ = [("struct_size", c_uint32), ("streams_open", c_int32), ("frames_done", c_int64),
                ("batches", c_int64), ("mean_batch_frames", ctypes.c_double),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("max_latency_s", ctypes.c_double), ("mpix_frames_per_s", ctypes.c_double),
                ("device_bytes_used", c_uint64), ("device_budget", c_uint64)]


FGS_DTYPE_F32, FGS_DTYPE_U32, FGS_DTYPE_U16 = 1, 2, 3


class fgs_state_field(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("index", c_int32), ("sub", c_int32), ("dtype", c_int32),
                ("elem_bytes", c_int32), ("base", c_void_p), ("pixel_stride", c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FgsError(-1, f"{LIB_PATH} is not built (run python -m paper_2002_00250_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    S = c_int32
    sig = {
        "fgs_abi_version": (c_int32, []),
        "fgs_status_str": (c_char_p, [c_int32]),
        "fgs_last_error": (c_char_p, []),
        "fgs_gmm_params_default": (S, [POINTER(fgs_gmm_params)]),
        "fgs_pbas_params_default": (S, [POINTER(fgs_pbas_params)]),
        "fgs_create": (S, [c_int32, c_int32, c_int32, c_void_p, c_void_p, POINTER(c_void_p)]),
        "fgs_destroy": (S, [c_void_p]),
        "fgs_push_frame": (S, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_int32]),
        "fgs_push_frame_scaled": (S, [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_int32, c_int32, c_int32]),
        "fgs_push_frames": (S, [POINTER(c_void_p), c_int32, POINTER(c_void_p), POINTER(c_int64),
                                POINTER(c_void_p), POINTER(c_int64)]),
        "fgs_get_mask": (S, [c_void_p, c_void_p, c_int64, c_int32]),
        "fgs_mask_device_ptr": (S, [c_void_p, POINTER(c_void_p)]),
        "fgs_eval_accumulate": (S, [c_void_p, c_void_p, c_int64, c_int32]),
        "fgs_eval_read": (S, [c_void_p, POINTER(c_uint64), c_int32]),
        "fgs_state_size": (S, [c_void_p, POINTER(c_size_t)]),
        "fgs_get_state": (S, [c_void_p, POINTER(fgs_state_field), c_int32, POINTER(c_int32)]),
        "fgs_copy_state": (S, [c_void_p, c_void_p, c_size_t, c_int32]),
        "fgs_copy_state_noalloc": (S, [c_void_p, c_void_p, c_size_t, c_int32]),
        "fgs_set_state": (S, [c_void_p, c_void_p, c_size_t, c_int32]),
        "fgs_frame_index": (S, [c_void_p, POINTER(c_int64)]),
        "fgs_sync": (S, [c_void_p]),
        "fgs_stream": (S, [c_void_p, POINTER(c_void_p)]),
        "fgs_device_bytes": (S, [c_void_p, POINTER(c_size_t)]),
        "fgs_set_cache_policy": (S, [c_void_p, c_int32]),
        "fgs_gmm_window_create": (S, [c_int32, c_int32, c_int32, POINTER(fgs_gmm_params), c_int32, c_void_p,
                                      POINTER(c_void_p)]),
        "fgs_gmm_window_forward": (S, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
        "fgs_gmm_window_backward": (S, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
        "fgs_gmm_window_records": (S, [c_void_p, c_void_p, c_int32]),
        "fgs_gmm_window_destroy": (S, [c_void_p]),
        "fgs_server_now": (ctypes.c_double, []),
        "fgs_server_create": (S, [c_size_t, c_int32, POINTER(c_void_p)]),
        "fgs_server_open": (S, [c_void_p, c_int32, c_int32, c_int32, c_void_p, POINTER(c_int32)]),
        "fgs_server_submit": (S, [c_void_p, c_int32, c_void_p, c_void_p, ctypes.c_double, POINTER(c_uint64)]),
        "fgs_server_wait": (S, [c_void_p, c_uint64, c_void_p, POINTER(ctypes.c_double), c_int32]),
        "fgs_server_close": (S, [c_void_p, c_int32]),
        "fgs_server_get_stats": (S, [c_void_p, POINTER(fgs_server_stats)]),
        "fgs_server_reset_stats": (S, [c_void_p]),
        "fgs_server_destroy": (S, [c_void_p]),
        "fgs_philox4x32_10": (S, [c_uint64, c_void_p, c_void_p, c_int64, c_void_p]),
        "fgs_copy_probe": (S, [c_void_p, c_void_p, c_size_t, c_void_p]),
        "fgs_mix_probe": (S, [c_void_p, c_int64, c_int32, c_void_p]),
        "fgs_mask_median": (S, [c_void_p, c_int64, c_void_p, c_int64, c_int32, c_int32, c_int32, c_void_p]),
        "fgs_static_enable": (S, [c_void_p, c_int32]),
        "fgs_static_mask": (S, [c_void_p, c_void_p, c_int64, c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if lib.fgs_abi_version() != ABI_VERSION:
        raise FgsError(-1, f"{LIB_PATH} has ABI version {lib.fgs_abi_version()}, the binding expects "
                           f"{ABI_VERSION}: rebuild it (python -m paper_2002_00250_amd.build)")
    _lib = lib
    return lib


def lib():
    return _load()


def _check(status: int):
    if status != FGS_OK:
        msg = _load().fgs_last_error().decode(errors="replace")
        raise FgsError(status, msg)


# ---------------------------------------------------------------- C entry points
def fgs_abi_version() -> int:
    return _load().fgs_abi_version()


def fgs_status_str(s: int) -> str:
    return _load().fgs_status_str(s).decode()


def fgs_last_error() -> str:
    return _load().fgs_last_error().decode(errors="replace")


def fgs_gmm_params_default() -> fgs_gmm_params:
    p = fgs_gmm_params()
    _check(_load().fgs_gmm_params_default(byref(p)))
    return p


def fgs_pbas_params_default() -> fgs_pbas_params:
    p = fgs_pbas_params()
    _check(_load().fgs_pbas_params_default(byref(p)))
    return p


def fgs_create(algo: int, H: int, W: int, params=None, hip_stream: int | None = None) -> int:
    out = c_void_p()
    pp = byref(params) if params is not None else None
    _check(_load().fgs_create(algo, H, W, pp, c_void_p(hip_stream or 0), byref(out)))
    return out.value


def fgs_destroy(m: int) -> None:
    _check(_load().fgs_destroy(c_void_p(m)))


def fgs_push_frame(m: int, rgb: int, rgb_stride: int, depth: int, depth_stride: int, where: int) -> None:
    _check(_load().fgs_push_frame(c_void_p(m), c_void_p(rgb), rgb_stride, c_void_p(depth),
                                  depth_stride, where))


def fgs_push_frame_scaled(m: int, rgb: int, rgb_stride: int, depth: int, depth_stride: int, depth_H: int,
                          depth_W: int, where: int) -> None:
    _check(_load().fgs_push_frame_scaled(c_void_p(m), c_void_p(rgb), rgb_stride, c_void_p(depth),
                                         depth_stride, depth_H, depth_W, where))


def fgs_push_frames(models, rgb, rgb_stride, depth, depth_stride) -> None:
    """Raw call: sequences of model handles, device frame addresses and row strides."""
    n = len(models)
    ptrs = lambda xs: (c_void_p * n)(*[c_void_p(x) for x in xs])
    i64 = lambda xs: (c_int64 * n)(*xs)
    _check(_load().fgs_push_frames(ptrs(models), n, ptrs(rgb), i64(rgb_stride), ptrs(depth), i64(depth_stride)))


def push_frames(models, rgbs, depths) -> None:
    """One device frame to each of several Models created on the same stream (uint8
    [H, W, 3] and 16-bit [H, W] cuda tensors, each of its model's size), in as few
    launches as the models' kinds and classes allow; the same results as pushing each."""
    if not models:
        return
    if not (len(models) == len(rgbs) == len(depths)):
        raise ValueError("models, rgbs and depths differ in length")
    for m, r, d in zip(models, rgbs, depths):
        m._check_frame(r, d)
    m0 = models[0]
    m0._model_waits_for_torch()
    fgs_push_frames([m.handle for m in models], [r.data_ptr() for r in rgbs], [r.stride(0) for r in rgbs],
                    [d.data_ptr() for d in depths], [2 * d.stride(0) for d in depths])
    m0._torch_waits_for_model()


def fgs_get_mask(m: int, mask: int, stride: int, where: int) -> None:
    _check(_load().fgs_get_mask(c_void_p(m), c_void_p(mask), stride, where))


def fgs_mask_device_ptr(m: int) -> int:
    out = c_void_p()
    _check(_load().fgs_mask_device_ptr(c_void_p(m), byref(out)))
    return out.value


def fgs_eval_accumulate(m: int, gt: int, gt_stride: int, where: int) -> None:
    _check(_load().fgs_eval_accumulate(c_void_p(m), c_void_p(gt), gt_stride, where))


def fgs_eval_read(m: int, reset: bool = False) -> tuple:
    """(TP, TN, FP, FN) accumulated so far."""
    out = (c_uint64 * 4)()
    _check(_load().fgs_eval_read(c_void_p(m), out, 1 if reset else 0))
    return tuple(int(v) for v in out)


def fgs_static_enable(m: int, M: int) -> None:
    _check(_load().fgs_static_enable(c_void_p(m), M))


def fgs_static_mask(m: int, out: int, stride: int, where: int) -> None:
    _check(_load().fgs_static_mask(c_void_p(m), c_void_p(out), stride, where))


def fgs_state_size(m: int) -> int:
    out = c_size_t()
    _check(_load().fgs_state_size(c_void_p(m), byref(out)))
    return out.value


def fgs_get_state(m: int) -> list:
    """The model's state fields in place: [{name, index, sub, dtype, elem_bytes, base,
    pixel_stride}] (device addresses, borrowed; see include/fgs.h)."""
    n = c_int32()
    _check(_load().fgs_get_state(c_void_p(m), None, 0, byref(n)))
    arr = (fgs_state_field * n.value)()
    _check(_load().fgs_get_state(c_void_p(m), arr, n.value, byref(n)))
    return [dict(name=f.name.decode(), index=f.index, sub=f.sub, dtype=f.dtype, elem_bytes=f.elem_bytes,
                 base=f.base or 0, pixel_stride=f.pixel_stride) for f in arr]


def fgs_copy_state(m: int, dst: int, nbytes: int, where: int) -> None:
    _check(_load().fgs_copy_state(c_void_p(m), c_void_p(dst), nbytes, where))


def fgs_copy_state_noalloc(m: int, dst: int, nbytes: int, where: int) -> None:
    _check(_load().fgs_copy_state_noalloc(c_void_p(m), c_void_p(dst), nbytes, where))


FGS_NOALLOC_STAGING_BYTES = 64 << 20


def fgs_set_state(m: int, src: int, nbytes: int, where: int) -> None:
    _check(_load().fgs_set_state(c_void_p(m), c_void_p(src), nbytes, where))


def fgs_frame_index(m: int) -> int:
    out = c_int64()
    _check(_load().fgs_frame_index(c_void_p(m), byref(out)))
    return out.value


def fgs_sync(m: int) -> None:
    _check(_load().fgs_sync(c_void_p(m)))


def fgs_stream(m: int) -> int:
    out = c_void_p()
    _check(_load().fgs_stream(c_void_p(m), byref(out)))
    return out.value or 0


def fgs_device_bytes(m: int) -> int:
    out = c_size_t()
    _check(_load().fgs_device_bytes(c_void_p(m), byref(out)))
    return out.value


def fgs_set_cache_policy(m: int, policy: int) -> None:
    _check(_load().fgs_set_cache_policy(c_void_p(m), policy))


def fgs_gmm_window_create(T: int, H: int, W: int, params=None, checkpoint_every: int = 16,
                          hip_stream: int | None = None) -> int:
    out = c_void_p()
    pp = byref(params) if params is not None else None
    _check(_load().fgs_gmm_window_create(T, H, W, pp, checkpoint_every, c_void_p(hip_stream or 0), byref(out)))
    return out.value


def fgs_gmm_window_forward(w: int, theta: int, rgb: int, depth: int, Z: int, has_term: int) -> None:
    _check(_load().fgs_gmm_window_forward(c_void_p(w), c_void_p(theta), c_void_p(rgb), c_void_p(depth),
                                          c_void_p(Z), c_void_p(has_term)))


def fgs_gmm_window_backward(w: int, theta: int, rgb: int, depth: int, dZ: int, dtheta: int) -> None:
    _check(_load().fgs_gmm_window_backward(c_void_p(w), c_void_p(theta), c_void_p(rgb), c_void_p(depth),
                                           c_void_p(dZ), c_void_p(dtheta)))


def fgs_gmm_window_records(w: int, out: int, where: int) -> None:
    _check(_load().fgs_gmm_window_records(c_void_p(w), c_void_p(out), where))


def fgs_gmm_window_destroy(w: int) -> None:
    _check(_load().fgs_gmm_window_destroy(c_void_p(w)))


def fgs_server_now() -> float:
    return _load().fgs_server_now()


def fgs_server_create(hbm_budget_bytes: int, max_streams: int) -> int:
    out = c_void_p()
    _check(_load().fgs_server_create(hbm_budget_bytes, max_streams, byref(out)))
    return out.value


def fgs_server_open(srv: int, algo: int, H: int, W: int, params=None) -> int:
    out = c_int32()
    pp = ctypes.cast(byref(params), c_void_p) if params is not None else None
    _check(_load().fgs_server_open(c_void_p(srv), algo, H, W, pp, byref(out)))
    return out.value


def fgs_server_submit(srv: int, stream_id: int, rgb: int, depth: int, t_arrival_s: float = 0.0) -> int:
    out = c_uint64()
    _check(_load().fgs_server_submit(c_void_p(srv), stream_id, c_void_p(rgb), c_void_p(depth), t_arrival_s,
                                     byref(out)))
    return out.value


def fgs_server_wait(srv: int, ticket: int, mask: int | None = None, timeout_ms: int = -1) -> float:
    lat = ctypes.c_double()
    _check(_load().fgs_server_wait(c_void_p(srv), ticket, c_void_p(mask or 0), byref(lat), timeout_ms))
    return lat.value


def fgs_server_close(srv: int, stream_id: int) -> None:
    _check(_load().fgs_server_close(c_void_p(srv), stream_id))


def fgs_server_get_stats(srv: int) -> dict:
    st = fgs_server_stats()
    st.struct_size = ctypes.sizeof(fgs_server_stats)
    _check(_load().fgs_server_get_stats(c_void_p(srv), byref(st)))
    return {k: getattr(st, k) for k, _ in fgs_server_stats._fields_ if k != "struct_size"}


def fgs_server_reset_stats(srv: int) -> None:
    _check(_load().fgs_server_reset_stats(c_void_p(srv)))


def fgs_server_destroy(srv: int) -> None:
    _check(_load().fgs_server_destroy(c_void_p(srv)))


def fgs_philox4x32_10(seed: int, ctr: int, out: int, n: int, hip_stream: int | None = None) -> None:
    _check(_load().fgs_philox4x32_10(seed, c_void_p(ctr), c_void_p(out), n, c_void_p(hip_stream or 0)))


def fgs_copy_probe(src: int, dst: int, nbytes: int, hip_stream: int | None = None) -> None:
    _check(_load().fgs_copy_probe(c_void_p(src), c_void_p(dst), nbytes, c_void_p(hip_stream or 0)))


def fgs_mix_probe(planes: int, npix: int, mode: int, hip_stream: int | None = None) -> None:
    _check(_load().fgs_mix_probe(c_void_p(planes), npix, mode, c_void_p(hip_stream or 0)))


def fgs_mask_median(src: int, src_stride: int, dst: int, dst_stride: int, H: int, W: int, radius: int,
                    hip_stream: int | None = None) -> None:
    _check(_load().fgs_mask_median(c_void_p(src), src_stride, c_void_p(dst), dst_stride, H, W, radius,
                                   c_void_p(hip_stream or 0)))


def median_mask(mask, radius: int, out=None):
    """Median post-filter of a binary device mask (uint8 [H, W] tensor on the GPU, rows
    contiguous): 255 where more than half of the (2r+1)^2 window is nonzero, border pixels
    replicated.  Runs on torch's current stream; returns `out` (allocated if None)."""
    import torch
    for name, t in (("mask", mask), ("out", out)):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.uint8 or t.dim() != 2:
            raise ValueError(f"{name} must be a uint8 [H, W] tensor on the GPU")
        if t.shape[1] > 1 and t.stride(1) != 1:
            raise ValueError(f"{name} rows must be contiguous")
        if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
            raise ValueError(f"{name} rows must not overlap (row stride {t.stride(0)} < width {t.shape[1]})")
    if out is None:
        out = torch.empty(mask.shape, dtype=torch.uint8, device=mask.device)
    elif tuple(out.shape) != tuple(mask.shape):
        raise ValueError("out must have the mask's shape")
    H, W = mask.shape

    def row_stride(t):   # one row: any stride >= W describes it
        return t.stride(0) if H > 1 else W
    stream = torch.cuda.current_stream(mask.device).cuda_stream
    fgs_mask_median(mask.data_ptr(), row_stride(mask), out.data_ptr(), row_stride(out), H, W, radius, stream)
    return out


# ---------------------------------------------------------------- state layout
def unpack_state(blob: np.ndarray) -> dict:
    """Split a serialised state (see fgs_copy_state) into named numpy planes."""
    b = np.ascontiguousarray(blob).view(np.uint8)
    hdr = b[:STATE_HEADER_BYTES]
    magic, version, algo = (int(v) for v in hdr[:12].view(np.uint32))
    H, W, A, B, flags = (int(v) for v in hdr[12:32].view(np.int32))
    frames = int(hdr[32:40].view(np.int64)[0])
    seed = int(hdr[40:48].view(np.uint64)[0])
    if magic != 0x53534746:
        raise ValueError("not an fgs state blob")
    pay = b[STATE_HEADER_BYTES:]
    n = H * W
    out = dict(algo=algo, H=H, W=W, t=frames, seed=seed)
    if algo == FGS_GMM:
        Kc, Kd = A, B
        f = pay.view(np.float32)
        o = 0

        def take(k, shape):
            nonlocal o
            a = f[o:o + k * n].reshape(shape)
            o += k * n
            return a
        diag = bool(flags & 1)   # per-channel colour variances
        out.update(Kc=Kc, Kd=Kd, w_c=take(Kc, (Kc, H, W)), mu_c=take(3 * Kc, (Kc, 3, H, W)),
                   v_c=take(3 * Kc, (Kc, 3, H, W)) if diag else take(Kc, (Kc, H, W)),
                   w_d=take(Kd, (Kd, H, W)), mu_d=take(Kd, (Kd, H, W)), v_d=take(Kd, (Kd, H, W)))
    elif flags & 2:   # PBAS with gradient-magnitude samples
        N = A
        u32 = pay[:2 * N * n * 4].view(np.uint32)
        out.update(N=N, gradient=True, samples=u32[:N * n].reshape(N, H, W),
                   gsamples=u32[N * n:].reshape(N, H, W))
        f = pay[2 * N * n * 4:(6 * N + 12) * n * 4].view(np.float32)
        out.update(dhist=f[:4 * N * n].reshape(N, 4, H, W), R=f[4 * N * n:(4 * N + 4) * n].reshape(4, H, W),
                   T=f[(4 * N + 4) * n:(4 * N + 8) * n].reshape(4, H, W),
                   S=f[(4 * N + 8) * n:(4 * N + 12) * n].reshape(4, H, W))
        out["gsum"] = pay[(6 * N + 12) * n * 4:].copy().view(np.uint64)
    else:
        N = A
        u32 = pay[:2 * N * n * 4].view(np.uint32)
        out.update(N=N, samples=u32[:N * n].reshape(N, H, W), dhist=u32[N * n:].reshape(N, H, W))
        rt = pay[2 * N * n * 4:2 * N * n * 4 + 8 * n * 4].view(np.float32)
        out.update(R=rt[:4 * n].reshape(4, H, W), T=rt[4 * n:].reshape(4, H, W))
        out.update(S=pay[2 * N * n * 4 + 8 * n * 4:].view(np.uint16).reshape(4, H, W))
    return out


def pack_state(st: dict) -> np.ndarray:
    """Inverse of unpack_state for a dict with the same keys."""
    hdr = np.zeros(STATE_HEADER_BYTES, np.uint8)
    algo = st["algo"]
    A, B = (st["Kc"], st["Kd"]) if algo == FGS_GMM else (st["N"], 0)
    hdr[:12] = np.array([0x53534746, 1, algo], np.uint32).view(np.uint8)
    flags = (1 if algo == FGS_GMM and np.ndim(st["v_c"]) == 4 else 0) | (2 if st.get("gradient") else 0)
    hdr[12:32] = np.array([st["H"], st["W"], A, B, flags], np.int32).view(np.uint8)
    hdr[32:40] = np.array([st["t"]], np.int64).view(np.uint8)
    hdr[40:48] = np.array([st.get("seed", 0)], np.uint64).view(np.uint8)
    if algo == FGS_GMM:
        parts = [np.asarray(st[k], np.float32).ravel() for k in ("w_c", "mu_c", "v_c", "w_d", "mu_d", "v_d")]
    elif st.get("gradient"):
        parts = [np.asarray(st["samples"], np.uint32).ravel(), np.asarray(st["gsamples"], np.uint32).ravel(),
                 np.asarray(st["dhist"], np.float32).ravel(), np.asarray(st["R"], np.float32).ravel(),
                 np.asarray(st["T"], np.float32).ravel(), np.asarray(st["S"], np.float32).ravel(),
                 np.asarray(st["gsum"], np.uint64).ravel()]
    else:
        parts = [np.asarray(st["samples"], np.uint32).ravel(), np.asarray(st["dhist"], np.uint32).ravel(),
                 np.asarray(st["R"], np.float32).ravel(), np.asarray(st["T"], np.float32).ravel(),
                 np.asarray(st["S"], np.uint16).ravel()]
    return np.concatenate([hdr] + [p.view(np.uint8) for p in parts])


# ---------------------------------------------------------------- convenience
class Model:
    """A background model on the current GPU.  Frames are torch tensors (device or host)
    or numpy arrays; ``rgb`` [H, W, 3] uint8, ``depth`` [H, W] uint16 (torch: int16 view
    or uint16).

    The model runs on its own stream (or the one given).  Device tensors are ordered with
    torch's current stream: the model's stream waits for the work queued there before a
    call that reads or writes a tensor, and torch's current stream then waits for the
    model, so a tensor the model wrote is ready and one it read may be reused or freed."""

    def __init__(self, algo: int, H: int, W: int, params=None, stream=None):
        import torch
        self._torch = torch
        self.algo, self.H, self.W = algo, H, W
        self.params = params
        handle = stream.cuda_stream if stream is not None else 0
        self.handle = fgs_create(algo, H, W, params, handle)
        self._mask_ptr = fgs_mask_device_ptr(self.handle)
        self._ext = None

    @property
    def mask_ptr(self) -> int:
        """Device address of the model's mask (H rows of W bytes, rows W apart), rewritten
        by every push in the model's stream order (fgs_mask_device_ptr)."""
        return self._mask_ptr

    def _model_stream(self):
        if self._ext is None:
            self._ext = self._torch.cuda.ExternalStream(fgs_stream(self.handle))
        return self._ext

    def _model_waits_for_torch(self):
        self._model_stream().wait_stream(self._torch.cuda.current_stream())

    def _torch_waits_for_model(self):
        self._torch.cuda.current_stream().wait_stream(self._model_stream())

    def close(self):
        if getattr(self, "handle", None):
            self._ext = None              # wraps the model's stream, destroyed next
            fgs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptr_where(x):
        if isinstance(x, np.ndarray):
            return x.ctypes.data, FGS_MEM_HOST
        return x.data_ptr(), (FGS_MEM_DEVICE if x.is_cuda else FGS_MEM_HOST)

    def _check_tensors(self, rgb, depth):
        torch = self._torch
        if rgb.dtype != torch.uint8 or rgb.dim() != 3 or rgb.shape[2] != 3 or \
                rgb.stride(2) != 1 or rgb.stride(1) != 3:
            raise ValueError("rgb must be uint8 [H, W, 3] with packed pixels (rows may be strided)")
        if depth.dtype not in (torch.int16, getattr(torch, "uint16", torch.int16)) or \
                depth.dim() != 2 or depth.stride(1) != 1:
            raise ValueError("depth must be 16-bit [H, W] with packed pixels (rows may be strided)")

    def _check_frame(self, rgb, depth):
        """A device frame of this model's size, for push_frames."""
        torch = self._torch
        if not isinstance(rgb, torch.Tensor) or not isinstance(depth, torch.Tensor) or \
                not rgb.is_cuda or not depth.is_cuda:
            raise ValueError("push_frames takes cuda tensors")
        self._check_tensors(rgb, depth)
        if tuple(rgb.shape[:2]) != (self.H, self.W) or tuple(depth.shape) != (self.H, self.W):
            raise ValueError(f"frames must be {(self.H, self.W)} for this model")

    def push(self, rgb, depth):
        """Push one frame; a depth map of another size than rgb is upscaled to it."""
        if isinstance(rgb, np.ndarray):
            rgb = np.ascontiguousarray(rgb, np.uint8)
            depth = np.ascontiguousarray(depth, np.uint16)
        else:
            self._check_tensors(rgb, depth)
        if tuple(rgb.shape[:2]) != (self.H, self.W):
            raise ValueError(f"rgb is {tuple(rgb.shape[:2])}, the model is {(self.H, self.W)}")
        pr, wr = self._ptr_where(rgb)
        pd, wd = self._ptr_where(depth)
        if wr != wd:
            raise ValueError("rgb and depth must both be host or both be device memory")
        rs = rgb.stride(0) if not isinstance(rgb, np.ndarray) else rgb.strides[0]
        ds = (depth.stride(0) * 2) if not isinstance(depth, np.ndarray) else depth.strides[0]
        dh, dw = int(depth.shape[0]), int(depth.shape[1])
        if wr == FGS_MEM_DEVICE:
            self._model_waits_for_torch()
        if (dh, dw) == (self.H, self.W):
            fgs_push_frame(self.handle, pr, rs, pd, ds, wr)
        else:
            fgs_push_frame_scaled(self.handle, pr, rs, pd, ds, dh, dw, wr)
        if wr == FGS_MEM_DEVICE:
            # torch's stream may reuse the frames' memory only after the model has read them
            # (no record_stream: the model's stream can be destroyed before the tensors are)
            self._torch_waits_for_model()

    def mask_host(self) -> np.ndarray:
        out = np.empty((self.H, self.W), np.uint8)
        fgs_get_mask(self.handle, out.ctypes.data, self.W, FGS_MEM_HOST)
        return out

    def eval_accumulate(self, gt) -> None:
        """Add the confusion counts of the current mask against gt (uint8 [H, W], nonzero =
        foreground; numpy array or cuda tensor) to the model's device counters."""
        if isinstance(gt, np.ndarray):
            g = np.ascontiguousarray(gt, np.uint8)
            fgs_eval_accumulate(self.handle, g.ctypes.data, g.strides[0], FGS_MEM_HOST)
        else:
            self._check_plane(gt, "gt")
            self._model_waits_for_torch()
            fgs_eval_accumulate(self.handle, gt.data_ptr(), gt.stride(0), FGS_MEM_DEVICE)
            self._torch_waits_for_model()

    def static_enable(self, M: int) -> None:
        """Static-object detection: 255 where the mask was foreground in each of the last
        M frames (fgs_static_enable; M = 0 turns it off)."""
        fgs_static_enable(self.handle, M)

    def static_mask_host(self) -> np.ndarray:
        out = np.empty((self.H, self.W), np.uint8)
        fgs_static_mask(self.handle, out.ctypes.data, self.W, FGS_MEM_HOST)
        return out

    def eval_read(self, reset: bool = False) -> tuple:
        """(TP, TN, FP, FN) accumulated since creation or the last reset."""
        return fgs_eval_read(self.handle, reset)

    def _check_plane(self, t, name):
        """A uint8 [H, W] cuda tensor whose rows are contiguous bytes (rows may be strided)."""
        torch = self._torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8 or \
                tuple(t.shape) != (self.H, self.W) or (self.W > 1 and t.stride(1) != 1):
            raise ValueError(f"{name} must be a uint8 [{self.H}, {self.W}] cuda tensor with contiguous rows")

    def mask_into(self, out) -> None:
        """Device-to-device copy of the latest mask into a uint8 [H, W] cuda tensor."""
        self._check_plane(out, "out")
        self._model_waits_for_torch()
        fgs_get_mask(self.handle, out.data_ptr(), out.stride(0), FGS_MEM_DEVICE)
        self._torch_waits_for_model()

    def state_blob(self) -> np.ndarray:
        n = fgs_state_size(self.handle)
        out = np.empty(n, np.uint8)
        fgs_copy_state(self.handle, out.ctypes.data, n, FGS_MEM_HOST)
        return out

    def state(self) -> dict:
        return unpack_state(self.state_blob())

    def set_state(self, st) -> None:
        blob = st if isinstance(st, np.ndarray) else pack_state(st)
        blob = np.ascontiguousarray(blob, np.uint8)
        fgs_set_state(self.handle, blob.ctypes.data, blob.size, FGS_MEM_HOST)

    @property
    def t(self) -> int:
        return fgs_frame_index(self.handle)

    def sync(self):
        fgs_sync(self.handle)

    @property
    def stream_handle(self) -> int:
        return fgs_stream(self.handle)
