"""Pins for the PBAS oracle's gradient-magnitude variant (reading R-23 of the base PBAS
feature that Sec. 3.2's method leaves out; opt-in).

Checked against: hand-derived Sobel magnitudes (tests/golden), scipy's Sobel filter with a
replicated border, the plain variant where the variant must reduce to it (alpha = 0, or
spatially flat frames), a brute-force per-pixel implementation written separately from
the vectorised oracle (loops over pixels, channels and samples in float32 scalars, the
neighbour writes gathered at their destinations), and invariants (sample provenance, S
tracking the sum of D)."""
import json
import os

import numpy as np
import pytest
from scipy import ndimage

from oracle.pbas import NB_DX, NB_DY, PbasParams, PbasRef, pbas_draws, sobel_l1_magnitude
from synth import Scene, preset

GOLD = os.path.join(os.path.dirname(__file__), "golden", "pbas_gradient_cases.json")


def test_sobel_hand_derived():
    for c in json.load(open(GOLD))["cases"]:
        got = sobel_l1_magnitude(np.array(c["plane"], np.uint8))
        assert got.tolist() == c["m"], c["note"]


def test_sobel_matches_scipy_with_replicated_border():
    rng = np.random.default_rng(5)
    for H, W in ((1, 1), (1, 9), (8, 1), (13, 17), (32, 40)):
        plane = rng.integers(0, 256, (H, W), dtype=np.uint8)
        x = plane.astype(np.int32)
        gx = ndimage.sobel(x, axis=1, mode="nearest")
        gy = ndimage.sobel(x, axis=0, mode="nearest")
        np.testing.assert_array_equal(sobel_l1_magnitude(plane), (np.abs(gx) + np.abs(gy)) >> 3)


def _frames_flashing(H, W, n, seed, flat_every=5):
    """Random textured frames whose contrast changes from frame to frame (so consecutive
    gradient means differ), every flat_every-th frame flat (mean 0), depth with holes."""
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 256, (H, W, 3))
    out = []
    for t in range(n):
        if t % flat_every == flat_every - 1:
            rgb = np.full((H, W, 3), rng.integers(0, 256), np.int64)
        else:
            c = rng.uniform(0.2, 1.0)
            rgb = 128 + c * (base - 128) + rng.normal(0, 6, (H, W, 3))
        D = rng.integers(1200, 3200, (H, W))
        D[rng.random((H, W)) < 0.1] = 0
        out.append((np.clip(np.rint(rgb), 0, 255).astype(np.uint8), D.astype(np.uint16)))
    return out


def test_alpha_zero_is_the_plain_variant():
    # w = 0 drops the gradient term: dist = |v - B^v| as in the plain variant, whose masks,
    # samples, R, T, D and S the variant must then reproduce (D and S as floats)
    cfg = preset("pbas_640x480", H=24, W=31)
    sc = Scene(cfg)
    a = PbasRef(24, 31, PbasParams(N=6, gradient=True, grad_alpha=0.0, seed=3))
    b = PbasRef(24, 31, PbasParams(N=6, seed=3))
    for t in range(40):
        rgb, D, _ = sc.frame(t)
        np.testing.assert_array_equal(a.step(rgb, D), b.step(rgb, D), err_msg=f"t={t}")
    np.testing.assert_array_equal(a.samples, b.samples)
    np.testing.assert_array_equal(a.R, b.R)
    np.testing.assert_array_equal(a.T, b.T)
    np.testing.assert_array_equal(a.D, b.D.astype(np.float32))
    np.testing.assert_array_equal(a.S, b.S.astype(np.float32))


def test_flat_frames_are_the_plain_variant_for_any_alpha():
    # frames constant over the image: every m = 0, every gradient distance 0
    rng = np.random.default_rng(2)
    a = PbasRef(6, 8, PbasParams(N=4, gradient=True, grad_alpha=25.0, seed=4))
    b = PbasRef(6, 8, PbasParams(N=4, seed=4))
    for t in range(30):
        rgb = np.broadcast_to(rng.integers(0, 256, 3).astype(np.uint8), (6, 8, 3)).copy()
        D = np.full((6, 8), int(rng.integers(0, 3000)), np.uint16)
        np.testing.assert_array_equal(a.step(rgb, D), b.step(rgb, D), err_msg=f"t={t}")
    np.testing.assert_array_equal(a.samples, b.samples)
    assert not a.gsamples.any()
    np.testing.assert_array_equal(a.S, b.S.astype(np.float32))


# ------------------------------------------------------------ brute force
def _clamp(v, lo, hi):
    return lo if v < lo else (hi if v > hi else v)


def _magnitude(plane, y, x):
    H, W = plane.shape
    px = lambda yy, xx: int(plane[_clamp(yy, 0, H - 1), _clamp(xx, 0, W - 1)])
    gx = gy = 0
    for d, wgt in ((-1, 1), (0, 2), (1, 1)):
        gx += wgt * (px(y + d, x + 1) - px(y + d, x - 1))
        gy += wgt * (px(y + 1, x + d) - px(y - 1, x + d))
    return (abs(gx) + abs(gy)) >> 3


class _Brute:
    """The variant pixel by pixel in float32 scalars (a separate restatement of R-23 over
    the base rules: fill, classify, self-update, neighbour update gathered at the
    destination, R and T)."""

    def __init__(self, H, W, p):
        self.H, self.W, self.p = H, W, p
        N = p.N
        self.v = np.zeros((N, H, W, 4), np.int64)
        self.m = np.zeros((N, H, W, 3), np.int64)
        self.D = np.zeros((N, H, W, 4), np.float32)
        self.S = np.zeros((H, W, 4), np.float32)
        self.R = np.zeros((H, W, 4), np.float32)
        self.T = np.full((H, W, 4), np.float32(p.T_lower), np.float32)
        for j in range(4):
            self.R[..., j] = np.float32(p.R_lower[j])
        self.prev_sum = [0, 0, 0]
        self.t = 0

    def step(self, I, valid):
        p, H, W, N = self.p, self.H, self.W, self.p.N
        f = np.float32
        M = np.zeros((H, W, 3), np.int64)
        for j in range(3):
            for y in range(H):
                for x in range(W):
                    M[y, x, j] = _magnitude(I[..., j], y, x)
        sums = [int(M[..., j].sum()) for j in range(3)]
        if self.t < N:
            self.v[self.t] = I
            self.m[self.t] = M
            self.prev_sum, self.t = sums, self.t + 1
            return np.zeros((H, W), np.uint8)
        wj = [f(p.grad_alpha) / max(f(float(s)) / f(H * W), f(1.0)) for s in self.prev_sum]
        w0, w1 = pbas_draws(H, W, self.t, p.seed)
        mask = np.zeros((H, W), np.uint8)
        Fm = np.zeros((H, W, 4), bool)
        dmin = np.zeros((H, W, 4), np.float32)
        for y in range(H):
            for x in range(W):
                for j in range(4):
                    if j == 3 and not valid[y, x]:
                        continue
                    cnt, best = 0, None
                    for k in range(N):
                        if j == 3 and self.v[k, y, x, 3] == 0:
                            continue
                        dv = f(abs(int(self.v[k, y, x, j]) - int(I[y, x, j])))
                        d = dv if j == 3 else f(wj[j] * f(abs(int(self.m[k, y, x, j]) - int(M[y, x, j])))) + dv
                        cnt += 1 if d < self.R[y, x, j] else 0
                        best = d if best is None or d < best else best
                    dmin[y, x, j] = f(255) if best is None else best
                    Fm[y, x, j] = cnt < p.min_matches
                    if Fm[y, x, j]:
                        mask[y, x] = 255
        T_prev = self.T.copy()
        fires = np.zeros((H, W, 4), bool)
        for y in range(H):
            for x in range(W):
                for j in range(4):
                    if (j == 3 and not valid[y, x]) or Fm[y, x, j]:
                        continue
                    a0, a1 = int(w0[y, x, j]), int(w1[y, x, j])
                    if f(a0 >> 16) * f(1 / 65536) * T_prev[y, x, j] < f(1):
                        k = ((a0 & 0xFFFF) * N) >> 16
                        self.v[k, y, x, j] = I[y, x, j]
                        if j < 3:
                            self.m[k, y, x, j] = M[y, x, j]
                        self.S[y, x, j] = f(f(self.S[y, x, j] - self.D[k, y, x, j]) + dmin[y, x, j])
                        self.D[k, y, x, j] = dmin[y, x, j]
                    fires[y, x, j] = f(a1 >> 16) * f(1 / 65536) * T_prev[y, x, j] < f(1)
        # neighbour writes, gathered: every pixel collects the writes aimed at it
        for y in range(H):
            for x in range(W):
                for oy in (-1, 0, 1):
                    for ox in (-1, 0, 1):
                        sy, sx = y + oy, x + ox
                        if (ox, oy) == (0, 0) or not (0 <= sy < H and 0 <= sx < W):
                            continue
                        for j in range(4):
                            a1 = int(w1[sy, sx, j])
                            d = (a1 >> 13) & 7
                            if not fires[sy, sx, j] or (sx + NB_DX[d], sy + NB_DY[d]) != (x, y):
                                continue
                            if j == 3 and not valid[y, x]:
                                continue
                            k = ((a1 & 0x1FFF) * N) >> 13
                            self.v[k, y, x, j] = I[y, x, j]
                            if j < 3:
                                self.m[k, y, x, j] = M[y, x, j]
        for y in range(H):
            for x in range(W):
                for j in range(4):
                    if j == 3 and not valid[y, x]:
                        continue
                    dbar = self.S[y, x, j] / f(N)
                    r = self.R[y, x, j]
                    with np.errstate(divide="ignore"):
                        r = r * (f(1) - f(p.R_incdec)) if r > dbar * f(p.R_scale) else r * (f(1) + f(p.R_incdec))
                        tt = (self.T[y, x, j] + f(p.T_inc) / dbar if Fm[y, x, j]
                              else self.T[y, x, j] - f(p.T_dec) / dbar)
                    self.R[y, x, j] = max(r, f(p.R_lower[j]))
                    self.T[y, x, j] = min(max(tt, f(p.T_lower)), f(p.T_upper))
        self.prev_sum, self.t = sums, self.t + 1
        return mask


@pytest.mark.parametrize("H,W,N,Tb,seed", [(7, 9, 4, (2.0, 200.0), 11), (5, 6, 3, (1.0, 1.0), 12)])
def test_matches_brute_force(H, W, N, Tb, seed):
    p = PbasParams(N=N, gradient=True, grad_alpha=10.0, T_lower=Tb[0], T_upper=Tb[1], seed=seed)
    ref = PbasRef(H, W, p)
    bf = _Brute(H, W, p)
    for t, (rgb, D) in enumerate(_frames_flashing(H, W, 22, seed)):
        m_ref = ref.step(rgb, D)
        I = ref.frame_value(rgb, D).astype(np.int64)
        m_bf = bf.step(I, D > 0)
        np.testing.assert_array_equal(m_ref, m_bf, err_msg=f"mask t={t}")
        np.testing.assert_array_equal(ref.samples, bf.v.astype(np.uint8), err_msg=f"samples t={t}")
        np.testing.assert_array_equal(ref.gsamples, bf.m.astype(np.uint8), err_msg=f"gsamples t={t}")
        for k in ("D", "S", "R", "T"):
            np.testing.assert_array_equal(getattr(ref, k), getattr(bf, k), err_msg=f"{k} t={t}")


def test_provenance_and_sum_of_d():
    cfg = preset("pbas_640x480", H=20, W=26)
    sc = Scene(cfg)
    p = PbasParams(N=8, gradient=True)
    ref = PbasRef(20, 26, p)
    seen = np.zeros((256, 20, 26, 3), bool)
    yy, xx = np.mgrid[0:20, 0:26]
    for t in range(60):
        rgb, D, _ = sc.frame(t)
        ref.step(rgb, D)
        M = np.stack([sobel_l1_magnitude(ref.frame_value(rgb, D)[..., j]) for j in range(3)], -1)
        for j in range(3):
            seen[M[..., j], yy, xx, j] = True
        # every magnitude in a sample is one this pixel has shown
        for k in range(min(p.N, t + 1)):
            for j in range(3):
                assert seen[ref.gsamples[k, :, :, j], yy, xx, j].all(), (t, k, j)
        # S follows the sum of D to float32 rounding
        assert np.all(np.abs(ref.S - ref.D.sum(0, dtype=np.float64)) <= 1e-4 * (1 + ref.D.sum(0)))
    assert np.all(ref.R >= np.array(p.R_lower, np.float32))
    assert np.all((ref.T >= p.T_lower) & (ref.T <= p.T_upper))
