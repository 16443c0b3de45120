"""GMM adjoint over a window of frames, as a torch.autograd.Function.

``GmmWindowFunction.apply(theta, rgb, depth, window)`` returns the pre-update scores
Z [T, H, W] (float32) and the term flags [T, H, W] (uint8) of a fresh RGB-D GMM run over
the window; its backward returns dL/dtheta for theta = (alpha, lambda, w_depth), with the
forward's discrete choices held fixed.  Both directions run in libfgs kernels
(fgs_gmm_window_forward / _backward); this module only orders them on torch streams.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fgs


class GmmWindow:
    """Device buffers (records, checkpoints, scratch) for T frames of H x W.  The records and
    checkpoints belong to the most recent forward; ``forwards`` counts them."""

    def __init__(self, T: int, H: int, W: int, params=None, checkpoint_every: int = 16, device=None):
        self.T, self.H, self.W = T, H, W
        self.forwards = 0
        self.device = torch.device(device or "cuda")
        self.stream = torch.cuda.Stream(self.device)
        self.handle = fgs.fgs_gmm_window_create(T, H, W, params, checkpoint_every, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            fgs.fgs_gmm_window_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rgb, depth):
        T, H, W = self.T, self.H, self.W
        if tuple(rgb.shape) != (T, H, W, 3) or rgb.dtype != torch.uint8 or not rgb.is_contiguous():
            raise ValueError("rgb must be a contiguous uint8 tensor [T, H, W, 3]")
        if tuple(depth.shape) != (T, H, W) or depth.dtype not in (torch.int16, torch.uint16) \
                or not depth.is_contiguous():
            raise ValueError("depth must be a contiguous 16-bit tensor [T, H, W]")

    def forward(self, theta: torch.Tensor, rgb: torch.Tensor, depth: torch.Tensor):
        self._check(rgb, depth)
        theta = theta.detach().to(torch.float32).contiguous()
        cur = torch.cuda.current_stream(self.device)
        Z = torch.empty((self.T, self.H, self.W), dtype=torch.float32, device=self.device)
        has = torch.empty((self.T, self.H, self.W), dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(cur)
        fgs.fgs_gmm_window_forward(self.handle, theta.data_ptr(), rgb.data_ptr(), depth.data_ptr(),
                                   Z.data_ptr(), has.data_ptr())
        cur.wait_stream(self.stream)
        for x in (theta, rgb, depth, Z, has):
            x.record_stream(self.stream)
        self.forwards += 1
        return Z, has

    def backward(self, theta: torch.Tensor, rgb: torch.Tensor, depth: torch.Tensor, dZ: torch.Tensor):
        self._check(rgb, depth)
        theta = theta.detach().to(torch.float32).contiguous()
        dZ = dZ.detach().to(torch.float32).contiguous()
        cur = torch.cuda.current_stream(self.device)
        out = torch.empty(3, dtype=torch.float64, device=self.device)
        self.stream.wait_stream(cur)
        fgs.fgs_gmm_window_backward(self.handle, theta.data_ptr(), rgb.data_ptr(), depth.data_ptr(),
                                    dZ.data_ptr(), out.data_ptr())
        cur.wait_stream(self.stream)
        for x in (theta, rgb, depth, dZ, out):
            x.record_stream(self.stream)
        return out

    def records(self) -> np.ndarray:
        out = np.empty((self.T, self.H, self.W), np.uint64)
        torch.cuda.current_stream(self.device).synchronize()
        fgs.fgs_gmm_window_records(self.handle, out.ctypes.data, fgs.FGS_MEM_HOST)
        return out


class GmmWindowFunction(torch.autograd.Function):
    """Z, has = apply(theta, rgb, depth, window).  Several applications may share a window
    (two windows of a sequence in one loss, a probe at another theta): the backward of an
    application whose records a later forward has overwritten first runs its own forward
    again on the saved inputs (the same kernels, so the same records), then the adjoint."""

    @staticmethod
    def forward(ctx, theta, rgb, depth, window: GmmWindow):
        Z, has = window.forward(theta, rgb, depth)
        ctx.save_for_backward(theta, rgb, depth)
        ctx.window = window
        ctx.forward_id = window.forwards
        ctx.mark_non_differentiable(has)
        return Z, has

    @staticmethod
    def backward(ctx, gZ, ghas):
        theta, rgb, depth = ctx.saved_tensors
        if ctx.window.forwards != ctx.forward_id:
            ctx.window.forward(theta, rgb, depth)
            ctx.forward_id = ctx.window.forwards
        d = ctx.window.backward(theta, rgb, depth, gZ)
        return d.to(theta.dtype), None, None, None


def window_bce_loss(Z: torch.Tensor, has: torch.Tensor, gt: torch.Tensor, t0: int = 1, tau: float = 1.0):
    """Mean BCE of sigmoid(Z/tau) against 0/255 ground truth over frames t >= t0 where Z has a term."""
    w = has[t0:].to(Z.dtype)
    y = (gt[t0:] != 0).to(Z.dtype)
    l = torch.nn.functional.binary_cross_entropy_with_logits(Z[t0:] / tau, y, weight=w, reduction="sum")
    return l / w.sum().clamp_min(1.0)
