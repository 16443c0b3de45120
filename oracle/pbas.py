"""RGB-D Pixel-Based Adaptive Segmenter: one classify-and-update step per frame.

Oracle (test infrastructure only).  Plain numpy, vectorised over pixels, one
loop over the N samples, the steps taken in the order of the method below.

What the paper fixes (Sec. 3.2) and what is read in
------------------------------------------------------
* PBAS (Hofmann et al. 2012, cited, not restated) keeps per pixel a buffer of
  N recent samples plus a second part, which the paper does not name; from the
  base method that is the adaptive decision threshold R, the adaptive update
  rate T and the history D of minimal decision distances.
* In the RGB-D variant one sample holds the RGB value and the depth value, and
  each component is segmented and updated on its own; depth takes part only
  where the sensor depth is > 0 (Sec. 3.2).  N = 20 in the authors' system.
  Samples are stored as 32-bit words, 8 bits per colour component and depth
  (Sec. 4.2), depth coded by ``oracle.depth.depth_q8``.
* Reading: four independent per-channel PBAS instances j in {R, G, B, D}; the
  pixel is foreground when any active channel is.  A depth byte of 0 in a
  sample means "no depth was recorded there": it never matches and is left out
  of d_min.

Per frame t and pixel x, for every active channel j (depth only if D(x) > 0):

  init       for t < N, sample slot t takes I(x, t); the mask is 0 and R, T,
             D, S stay at their initial values (R_lower, T_lower, 0, 0)
  classify   dist_k = |I_j - B_k,j|;  cnt = #{k : dist_k < R_j};
             d_min = min_k dist_k (255 if no sample);  F_j = cnt < #min
  draws      two Philox4x32-10 blocks per pixel and frame, counter
             (y*W + x, t, c, 0) for c = 0, 1, key = the 64-bit seed; word j of
             block c serves channel j.  From a word w: u = (w >> 16) / 2^16.
  self       if not F_j and u(w0_j) * T_j < 1 (T_j before this frame's update):
             k = ((w0_j & 0xFFFF) * N) >> 16;  B_k,j = I_j;
             S_j = S_j - D_k,j + d_min;  D_k,j = d_min
  neighbour  if not F_j and u(w1_j) * T_j < 1: the 8-neighbour y in direction
             (w1_j >> 13) & 7 (order: (-1,-1) (0,-1) (1,-1) (-1,0) (1,0)
             (-1,1) (0,1) (1,1) as (dx, dy)) gets slot
             k' = ((w1_j & 0x1FFF) * N) >> 13 of channel j set to y's own value
             I_j(y, t); skipped if y is outside the image, and for depth unless
             D(y) > 0
  R          d_bar = S_j / N;  R_j = R_j * (1 - R_inc/dec) if R_j > d_bar * R_scale
             else R_j * (1 + R_inc/dec);  R_j = max(R_j, R_lower,j)
  T          T_j = T_j + T_inc / d_bar if F_j else T_j - T_dec / d_bar
             (IEEE: d_bar = 0 gives +-inf), clamped to [T_lower, T_upper]

Every write into pixel y's samples during frame t carries y's own value at t,
and D, S are touched only by the pixel itself, so the result does not depend
on the order in which pixels are processed.  Classification of every pixel at
frame t sees the model as left by frame t-1.

Gradient-magnitude variant (``PbasParams.gradient``; opt-in, a reading of the base
method's second feature, which the paper's RGB-D variant does not use)
--------------------------------------------------------------------------------
The base PBAS adds to each sample the gradient magnitude of the pixel and measures
dist = alpha / mean_m * |m - B^m_k| + |v - B^v_k|, mean_m the average gradient
magnitude of the last observed frame.  Read here, for the colour channels only (the
depth channel keeps the value distance above):

  m_j        (|gx| + |gy|) >> 3 of channel j's plane of the current frame, gx, gy
             the 3x3 Sobel responses with the border replicated (an exact byte)
  mean_j     float32(float64(sum over the image of m_j)) / float32(H * W)
  w_j        float32(alpha) / max(mean_j of frame t-1, 1)   (float32)
  dist_k,j   w_j * |m_j - B^m_k,j| + |v_j - B^v_k,j|          (float32, in that order)
  d_min      float32; D holds float32 d_min; S = (S - D_k) + d_min (float32, in that
             order) on a self-update; R, T as above from d_bar = S / N
  samples    slot k of channel j holds (v, m); the fill frames, the self-update and
             the neighbour update write both (the neighbour its own v and m)
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .depth import DEPTH_MAX_MM, depth_q8
from .philox import philox4x32_10, seed_key

# 8-neighbourhood, indexed by the 3-bit direction field.
NB_DX = np.array([-1, 0, 1, -1, 1, -1, 0, 1], np.int64)
NB_DY = np.array([-1, -1, -1, 0, 0, 1, 1, 1], np.int64)

PBAS_DEFAULT_SEED = 0x2002_0025_0


@dataclass
class PbasParams:
    """Constants.  N from Sec. 3.2; the rest are the base method's published defaults,
    except the depth channel's R_lower (4 codes, about 16 cm), a reading."""
    N: int = 20
    min_matches: int = 2
    R_incdec: float = 0.05
    R_scale: float = 5.0
    T_inc: float = 1.0
    T_dec: float = 0.05
    T_lower: float = 2.0
    T_upper: float = 200.0
    R_lower: tuple = (18.0, 18.0, 18.0, 4.0)
    depth_max_mm: int = DEPTH_MAX_MM
    seed: int = PBAS_DEFAULT_SEED
    gradient: bool = False      # the gradient-magnitude variant (colour channels)
    grad_alpha: float = 10.0    # its weight alpha (the base method's default)


def sobel_l1_magnitude(plane: np.ndarray) -> np.ndarray:
    """Gradient magnitude of one 8-bit plane (reading of the base PBAS feature): the 3x3
    Sobel responses gx (right minus left column, rows weighted 1, 2, 1) and gy (bottom
    minus top row) with the border replicated, then (|gx| + |gy|) >> 3, a byte."""
    H, W = plane.shape
    P = np.pad(np.asarray(plane, np.int32), 1, mode="edge")

    def at(dy, dx):
        return P[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    gx = (at(-1, 1) + 2 * at(0, 1) + at(1, 1)) - (at(-1, -1) + 2 * at(0, -1) + at(1, -1))
    gy = (at(1, -1) + 2 * at(1, 0) + at(1, 1)) - (at(-1, -1) + 2 * at(-1, 0) + at(-1, 1))
    return ((np.abs(gx) + np.abs(gy)) >> 3).astype(np.uint8)


def gradient_mean(gsum, npix: int) -> np.ndarray:
    """Frame mean of the gradient magnitudes from their exact integer sums (float32)."""
    return np.asarray(gsum, np.uint64).astype(np.float64).astype(np.float32) / np.float32(npix)


def pbas_draws(H: int, W: int, t: int, seed: int, origin=None):
    """Philox words for frame t (R-17): (w0, w1), each uint32 [H, W, 4] (word j -> channel j).
    The counter's first word is the pixel's linear index y * W_img + x in the whole image;
    ``origin = (y0, x0, W_img)`` places this H x W array as a window of a larger image."""
    k0, k1 = seed_key(seed)
    if origin is None:
        pix = np.arange(H * W, dtype=np.uint64).reshape(H, W)
    else:
        y0, x0, W_img = origin
        ys = np.arange(y0, y0 + H, dtype=np.uint64)[:, None]
        xs = np.arange(x0, x0 + W, dtype=np.uint64)[None, :]
        pix = ys * np.uint64(W_img) + xs
    out = []
    for c in (0, 1):
        x = philox4x32_10(pix, np.uint64(t), np.uint64(c), np.uint64(0), k0, k1)
        out.append(np.stack(x, axis=-1))
    return out[0], out[1]


class PbasRef:
    """The RGB-D PBAS over an H x W image (Sec. 3.2: samples of RGB and depth, each
    component segmented and updated on its own, R-14).  ``step(rgb, depth) -> mask``."""

    def __init__(self, H: int, W: int, params: PbasParams | None = None, origin=None):
        """``origin = (y0, x0, W_img)``: this model is the window of rows y0.. and columns
        x0.. of a W_img-wide image, and draws that image's random numbers.  Writes that the
        image's pixels outside the window would send into it are not modelled, so only the
        window's outermost ring can differ from the whole image's model, and only in its
        samples."""
        self.p = params or PbasParams()
        self.H, self.W = H, W
        self.origin = origin
        N = self.p.N
        self.samples = np.zeros((N, H, W, 4), np.uint8)
        if self.p.gradient:
            if origin is not None:
                raise ValueError("the gradient variant needs the whole image (Sobel, frame mean)")
            self.gsamples = np.zeros((N, H, W, 3), np.uint8)
            self.D = np.zeros((N, H, W, 4), np.float32)
            self.S = np.zeros((H, W, 4), np.float32)
            self.gsum_prev = np.zeros(3, np.uint64)
        else:
            self.D = np.zeros((N, H, W, 4), np.uint8)
            self.S = np.zeros((H, W, 4), np.int64)
        self.R = np.broadcast_to(np.array(self.p.R_lower, np.float32), (H, W, 4)).copy()
        self.T = np.full((H, W, 4), np.float32(self.p.T_lower), np.float32)
        self.t = 0
        self.last_F = None
        self.last_draws = None

    def frame_value(self, rgb, depth) -> np.ndarray:
        """I(x, t): RGB bytes plus the depth code (0 where depth is invalid): the RGBD8
        sample word of Sec. 4.2 with the depth code of R-03."""
        I = np.empty((self.H, self.W, 4), np.uint8)
        I[..., :3] = rgb
        I[..., 3] = depth_q8(depth, self.p.depth_max_mm)
        return I

    def step(self, rgb: np.ndarray, depth: np.ndarray) -> np.ndarray:
        """One frame (Sec. 3.2): the fill phase for the first N frames (R-16), else the
        per-channel segmentation against the previous model (R-14, R-15), the self-update
        (R-18) and neighbour update (R-19) driven by the Philox words (R-17), and the R/T
        adaptation (R-20)."""
        if self.p.gradient:
            return self._step_gradient(rgb, depth)
        p = self.p
        H, W, N = self.H, self.W, p.N
        I = self.frame_value(rgb, depth)
        valid = np.asarray(depth) > 0
        active = np.ones((H, W, 4), np.bool_)
        active[..., 3] = valid

        if self.t < N:                      # initialisation: fill slot t
            self.samples[self.t] = I
            self.t += 1
            self.last_F = np.zeros((H, W, 4), np.bool_)
            return np.zeros((H, W), np.uint8)

        # Segmentation against the model left by frame t-1.
        Ii = I.astype(np.int16)
        cnt = np.zeros((H, W, 4), np.int64)
        dmin = np.full((H, W, 4), 255, np.int16)
        for k in range(N):
            s = self.samples[k]
            dist = np.abs(s.astype(np.int16) - Ii)
            filled = np.ones((H, W, 4), np.bool_)
            filled[..., 3] = s[..., 3] != 0
            cnt += filled & (dist < self.R)
            dmin = np.where(filled, np.minimum(dmin, dist), dmin)
        F = active & (cnt < p.min_matches)
        mask = np.where(F.any(axis=-1), 255, 0).astype(np.uint8)
        bg = active & ~F

        w0, w1 = pbas_draws(H, W, self.t, p.seed, self.origin)
        self.last_draws = (w0, w1)
        scale = np.float32(1.0 / 65536.0)
        T_prev = self.T

        # Self-update: a random sample and its d_min slot, with probability 1/T.
        u0 = (w0 >> np.uint32(16)).astype(np.float32) * scale
        upd = bg & (u0 * T_prev < np.float32(1.0))
        kself = (((w0 & np.uint32(0xFFFF)).astype(np.uint64) * np.uint64(N)) >> np.uint64(16)).astype(np.int64)
        ys, xs, js = np.nonzero(upd)
        ks = kself[ys, xs, js]
        self.samples[ks, ys, xs, js] = I[ys, xs, js]
        old = self.D[ks, ys, xs, js].astype(np.int64)
        dm = dmin[ys, xs, js].astype(np.int64)
        self.S[ys, xs, js] += dm - old
        self.D[ks, ys, xs, js] = dm.astype(np.uint8)

        # Neighbour update: a random neighbour's random sample takes the neighbour's own value.
        u1 = (w1 >> np.uint32(16)).astype(np.float32) * scale
        nb = bg & (u1 * T_prev < np.float32(1.0))
        direc = ((w1 >> np.uint32(13)) & np.uint32(7)).astype(np.int64)
        knb = (((w1 & np.uint32(0x1FFF)).astype(np.uint64) * np.uint64(N)) >> np.uint64(13)).astype(np.int64)
        ys, xs, js = np.nonzero(nb)
        d = direc[ys, xs, js]
        ny, nx = ys + NB_DY[d], xs + NB_DX[d]
        ok = (ny >= 0) & (ny < H) & (nx >= 0) & (nx < W)
        ys, xs, js, ny, nx = ys[ok], xs[ok], js[ok], ny[ok], nx[ok]
        ok = (js < 3) | valid[ny, nx]
        ys, xs, js, ny, nx = ys[ok], xs[ok], js[ok], ny[ok], nx[ok]
        self.samples[knb[ys, xs, js], ny, nx, js] = I[ny, nx, js]

        # Decision threshold and update rate.
        f = np.float32
        with np.errstate(divide="ignore"):
            dbar = self.S.astype(f) / f(N)
            R_new = np.where(self.R > dbar * f(p.R_scale),
                             self.R * (f(1) - f(p.R_incdec)), self.R * (f(1) + f(p.R_incdec)))
            R_new = np.maximum(R_new, np.array(p.R_lower, f))
            T_new = np.where(F, self.T + f(p.T_inc) / dbar, self.T - f(p.T_dec) / dbar)
        T_new = np.minimum(np.maximum(T_new, f(p.T_lower)), f(p.T_upper))
        self.R = np.where(active, R_new, self.R).astype(f)
        self.T = np.where(active, T_new, self.T).astype(f)
        self.last_F = F
        self.last_self = upd
        self.last_nb = nb
        self.t += 1
        return mask

    def _step_gradient(self, rgb: np.ndarray, depth: np.ndarray) -> np.ndarray:
        """One frame of the gradient-magnitude variant (module docstring): the steps of
        ``step`` in the same order, with (v, m) samples and float32 distances, D and S
        on the colour channels."""
        p = self.p
        H, W, N = self.H, self.W, p.N
        f = np.float32
        I = self.frame_value(rgb, depth)
        M = np.stack([sobel_l1_magnitude(I[..., j]) for j in range(3)], axis=-1)
        gsum = M.reshape(-1, 3).sum(axis=0, dtype=np.uint64)
        valid = np.asarray(depth) > 0
        active = np.ones((H, W, 4), np.bool_)
        active[..., 3] = valid

        if self.t < N:                      # initialisation: fill slot t
            self.samples[self.t] = I
            self.gsamples[self.t] = M
            self.gsum_prev = gsum
            self.t += 1
            self.last_F = np.zeros((H, W, 4), np.bool_)
            return np.zeros((H, W), np.uint8)

        # Segmentation against the model left by frame t-1, weights from frame t-1's mean.
        wgt = f(p.grad_alpha) / np.maximum(gradient_mean(self.gsum_prev, H * W), f(1.0))
        Ii = I.astype(np.int16)
        Mi = M.astype(np.int16)
        cnt = np.zeros((H, W, 4), np.int64)
        dmin = np.full((H, W, 4), np.inf, f)
        for k in range(N):
            s = self.samples[k]
            dv = np.abs(s.astype(np.int16) - Ii).astype(f)
            dm = np.abs(self.gsamples[k].astype(np.int16) - Mi).astype(f)
            dist = dv.copy()
            dist[..., :3] = wgt * dm + dv[..., :3]
            filled = np.ones((H, W, 4), np.bool_)
            filled[..., 3] = s[..., 3] != 0
            cnt += filled & (dist < self.R)
            dmin = np.where(filled, np.minimum(dmin, dist), dmin)
        dmin = np.where(np.isinf(dmin), f(255), dmin)      # a depth channel with no sample
        F = active & (cnt < p.min_matches)
        mask = np.where(F.any(axis=-1), 255, 0).astype(np.uint8)
        bg = active & ~F

        w0, w1 = pbas_draws(H, W, self.t, p.seed, self.origin)
        self.last_draws = (w0, w1)
        scale = f(1.0 / 65536.0)
        T_prev = self.T

        # Self-update: a random sample (value and magnitude) and its D slot, w.p. 1/T.
        u0 = (w0 >> np.uint32(16)).astype(f) * scale
        upd = bg & (u0 * T_prev < f(1.0))
        kself = (((w0 & np.uint32(0xFFFF)).astype(np.uint64) * np.uint64(N)) >> np.uint64(16)).astype(np.int64)
        ys, xs, js = np.nonzero(upd)
        ks = kself[ys, xs, js]
        self.samples[ks, ys, xs, js] = I[ys, xs, js]
        c = js < 3
        self.gsamples[ks[c], ys[c], xs[c], js[c]] = M[ys[c], xs[c], js[c]]
        old = self.D[ks, ys, xs, js]
        dm = dmin[ys, xs, js]
        self.S[ys, xs, js] = (self.S[ys, xs, js] - old) + dm
        self.D[ks, ys, xs, js] = dm

        # Neighbour update: a random neighbour's random sample takes its own value and
        # magnitude.
        u1 = (w1 >> np.uint32(16)).astype(f) * scale
        nb = bg & (u1 * T_prev < f(1.0))
        direc = ((w1 >> np.uint32(13)) & np.uint32(7)).astype(np.int64)
        knb = (((w1 & np.uint32(0x1FFF)).astype(np.uint64) * np.uint64(N)) >> np.uint64(13)).astype(np.int64)
        ys, xs, js = np.nonzero(nb)
        d = direc[ys, xs, js]
        ny, nx = ys + NB_DY[d], xs + NB_DX[d]
        ok = (ny >= 0) & (ny < H) & (nx >= 0) & (nx < W)
        ys, xs, js, ny, nx = ys[ok], xs[ok], js[ok], ny[ok], nx[ok]
        ok = (js < 3) | valid[ny, nx]
        ys, xs, js, ny, nx = ys[ok], xs[ok], js[ok], ny[ok], nx[ok]
        kk = knb[ys, xs, js]
        self.samples[kk, ny, nx, js] = I[ny, nx, js]
        c = js < 3
        self.gsamples[kk[c], ny[c], nx[c], js[c]] = M[ny[c], nx[c], js[c]]

        # Decision threshold and update rate, as in ``step``.
        with np.errstate(divide="ignore"):
            dbar = self.S / f(N)
            R_new = np.where(self.R > dbar * f(p.R_scale),
                             self.R * (f(1) - f(p.R_incdec)), self.R * (f(1) + f(p.R_incdec)))
            R_new = np.maximum(R_new, np.array(p.R_lower, f))
            T_new = np.where(F, self.T + f(p.T_inc) / dbar, self.T - f(p.T_dec) / dbar)
        T_new = np.minimum(np.maximum(T_new, f(p.T_lower)), f(p.T_upper))
        self.R = np.where(active, R_new, self.R).astype(f)
        self.T = np.where(active, T_new, self.T).astype(f)
        self.gsum_prev = gsum
        self.last_F = F
        self.last_self = upd
        self.last_nb = nb
        self.last_M = M
        self.t += 1
        return mask

    # State in the library's canonical plane order (see include/fgs.h).
    def state_planes(self) -> dict:
        """The state in the library's serialised plane order (fgs_copy_state's payload)."""
        if self.p.gradient:
            g4 = np.zeros(self.gsamples.shape[:-1] + (4,), np.uint8)
            g4[..., :3] = self.gsamples
            return dict(samples=np.ascontiguousarray(self.samples).view(np.uint32)[..., 0],
                        gsamples=g4.view(np.uint32)[..., 0],
                        dhist=np.moveaxis(self.D, -1, 1).copy(),
                        R=np.moveaxis(self.R, -1, 0).copy(), T=np.moveaxis(self.T, -1, 0).copy(),
                        S=np.moveaxis(self.S, -1, 0).copy(), gsum=self.gsum_prev.copy(), t=self.t)
        return dict(samples=np.ascontiguousarray(self.samples).view(np.uint32)[..., 0],
                    dhist=np.ascontiguousarray(self.D).view(np.uint32)[..., 0],
                    R=np.moveaxis(self.R, -1, 0).copy(), T=np.moveaxis(self.T, -1, 0).copy(),
                    S=np.moveaxis(self.S, -1, 0).astype(np.uint16), t=self.t)

    def set_state_planes(self, st: dict) -> None:
        """Replace the state from planes in that order (fgs_set_state's payload)."""
        N, H, W = self.p.N, self.H, self.W
        if self.p.gradient:
            self.samples = np.ascontiguousarray(st["samples"], np.uint32).view(np.uint8).reshape(N, H, W, 4).copy()
            g4 = np.ascontiguousarray(st["gsamples"], np.uint32).view(np.uint8).reshape(N, H, W, 4)
            self.gsamples = g4[..., :3].copy()
            self.D = np.moveaxis(np.asarray(st["dhist"], np.float32), 1, -1).copy()
            self.R = np.moveaxis(np.asarray(st["R"], np.float32), 0, -1).copy()
            self.T = np.moveaxis(np.asarray(st["T"], np.float32), 0, -1).copy()
            self.S = np.moveaxis(np.asarray(st["S"], np.float32), 0, -1).copy()
            self.gsum_prev = np.asarray(st["gsum"], np.uint64).copy()
            self.t = int(st["t"])
            return
        self.samples = np.ascontiguousarray(st["samples"], np.uint32).view(np.uint8).reshape(N, H, W, 4).copy()
        self.D = np.ascontiguousarray(st["dhist"], np.uint32).view(np.uint8).reshape(N, H, W, 4).copy()
        self.R = np.moveaxis(np.asarray(st["R"], np.float32), 0, -1).copy()
        self.T = np.moveaxis(np.asarray(st["T"], np.float32), 0, -1).copy()
        self.S = np.moveaxis(np.asarray(st["S"]), 0, -1).astype(np.int64)
        self.t = int(st["t"])
