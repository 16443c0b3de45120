"""Seeded synthetic RGB-D sequences with ground-truth foreground masks.

This module only *draws inputs*: it holds none of the background-model
arithmetic (no depth quantisation, no distances, no model update).  The CPU
oracle and the GPU library both consume its frames, so it is the one piece of
code they share.

The scenes stand in for the RealSense recordings and the SBM-RGBD sequences
the paper evaluates on (Sec. 5: illumination changes, colour camouflage,
depth camouflage, shadows), neither of which is available here.  What is
drawn:

* a static textured RGB background (mean 128, three oriented sinusoids with
  periods 8-64 px and amplitude 20 each, a fixed per-pixel U(-20, 20)
  texture), clipped to [0, 255];
* two depth planes in millimetres, 1500 mm on the left half and 3000 mm on
  the right half (sensor range 0.1-10 m, Sec. 4.1);
* ``n_objects`` textured rectangles at 900 mm, sides U{40..80}*(W/320) px,
  moving at constant speed 1-4*(W/320) px/frame and bouncing off the borders;
* optional global illumination ramp (a triangle wave between -30 and +30 over
  100 frames, period 200), optional colour-camouflaged rectangle (RGB equal to
  the background, depth 600 mm nearer) and optional shadows (the background
  RGB scaled by 0.6 in a copy of each rectangle shifted by (+0.15w, +0.10h),
  depth unchanged, not foreground);
* optionally, rectangles that stop moving at a given frame and stay (left objects, for
  static-object detection);
* per-frame noise: RGB + round(N(0, 3)), depth + round(N(0, 10 mm)) clipped to
  >= 1, then 2 % i.i.d. zero-depth holes (invalid depth, ground truth kept).

Every frame is a pure function of (config, t): the static part comes from
``SeedSequence([seed, 0])`` and frame t's noise from ``SeedSequence([seed, 1,
t])``, so any frame can be generated alone and in any order.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

__all__ = ["SceneConfig", "Scene", "PRESETS", "preset"]

DEFAULT_SEED = 200200250


@dataclass(frozen=True)
class SceneConfig:
    H: int
    W: int
    n_objects: int = 3
    illumination: bool = False
    camouflage: bool = False
    shadows: bool = False
    rgb_noise: float = 3.0
    depth_noise_mm: float = 10.0
    hole_frac: float = 0.02
    near_mm: int = 900
    planes_mm: tuple = (1500, 3000)
    camouflage_offset_mm: int = 600
    seed: int = DEFAULT_SEED
    stop_at: int = -1          # >= 0: the rectangles stop moving at this frame (left objects)

    def replace(self, **kw) -> "SceneConfig":
        return dataclasses.replace(self, **kw)


# The workloads the benchmarks and parity tests are quoted on.
PRESETS = {
    # GMM K=3 parity workload: 320x240, 3 rectangles.
    "gmm_320x240": SceneConfig(H=240, W=320, n_objects=3),
    # PBAS N=20 workload: 640x480, illumination ramp + colour-camouflaged object.
    "pbas_640x480": SceneConfig(H=480, W=640, n_objects=3, illumination=True,
                                camouflage=True),
    # Throughput workload at the D415/D435 depth resolution: 8 objects + shadows.
    "hd_1280x720": SceneConfig(H=720, W=1280, n_objects=8, shadows=True),
    # Adjoint workload: the 320x240 scene recipe at 640x480.
    "adjoint_640x480": SceneConfig(H=480, W=640, n_objects=3),
}


def preset(name: str, **overrides) -> SceneConfig:
    cfg = PRESETS[name]
    return cfg.replace(**overrides) if overrides else cfg


def _triangle(t: int, amp: float = 30.0, half_period: int = 100) -> float:
    """Triangle wave rising from -amp to +amp over ``half_period`` frames."""
    ph = t % (2 * half_period)
    if ph <= half_period:
        return -amp + 2.0 * amp * ph / half_period
    return amp - 2.0 * amp * (ph - half_period) / half_period


def _bounce(p0: float, v: float, t: int, span: float) -> float:
    """Position of a point moving at speed v inside [0, span], reflecting at the ends."""
    if span <= 0:
        return 0.0
    s = (p0 + v * t) % (2.0 * span)
    return s if s <= span else 2.0 * span - s


class Scene:
    """A deterministic RGB-D sequence: ``frame(t) -> (rgb u8[H,W,3], depth u16[H,W], gt u8[H,W])``."""

    def __init__(self, cfg: SceneConfig):
        self.cfg = cfg
        H, W = cfg.H, cfg.W
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg.seed, 0])))
        yy, xx = np.mgrid[0:H, 0:W].astype(np.float32)
        bg = np.full((H, W, 3), 128.0, np.float32)
        for _ in range(3):
            period = rng.uniform(8.0, 64.0)
            theta = rng.uniform(0.0, np.pi)
            phase = rng.uniform(0.0, 2.0 * np.pi, size=3)
            arg = (2.0 * np.pi / period) * (np.cos(theta) * xx + np.sin(theta) * yy)
            for c in range(3):
                bg[..., c] += 20.0 * np.sin(arg + phase[c])
        bg += rng.uniform(-20.0, 20.0, size=(H, W, 3)).astype(np.float32)
        self.bg_rgb = np.clip(bg, 0.0, 255.0).astype(np.float32)
        self.bg_depth = np.where(xx < W / 2.0, cfg.planes_mm[0], cfg.planes_mm[1]).astype(np.float32)

        scale = W / 320.0
        self.objects = []
        for _ in range(cfg.n_objects):
            w = max(1, min(W, int(round(int(rng.integers(40, 81)) * scale))))
            h = max(1, min(H, int(round(int(rng.integers(40, 81)) * scale))))
            colour = rng.integers(0, 256, size=3).astype(np.float32)
            tex = rng.uniform(-10.0, 10.0, size=(h, w, 3)).astype(np.float32)
            speed = rng.uniform(1.0, 4.0) * scale
            ang = rng.uniform(0.0, 2.0 * np.pi)
            x0 = rng.uniform(0.0, max(0.0, W - w))
            y0 = rng.uniform(0.0, max(0.0, H - h))
            self.objects.append(dict(w=w, h=h, rgb=np.clip(colour + tex, 0, 255),
                                     vx=speed * np.cos(ang), vy=speed * np.sin(ang),
                                     x0=x0, y0=y0))
        self.camo = None
        if cfg.camouflage:
            w = max(1, min(W, int(round(int(rng.integers(40, 81)) * scale))))
            h = max(1, min(H, int(round(int(rng.integers(40, 81)) * scale))))
            speed = rng.uniform(1.0, 4.0) * scale
            ang = rng.uniform(0.0, 2.0 * np.pi)
            self.camo = dict(w=w, h=h, vx=speed * np.cos(ang), vy=speed * np.sin(ang),
                             x0=rng.uniform(0.0, max(0.0, W - w)),
                             y0=rng.uniform(0.0, max(0.0, H - h)))

    def _pos(self, o, t):
        H, W = self.cfg.H, self.cfg.W
        if self.cfg.stop_at >= 0:
            t = min(t, self.cfg.stop_at)
        x = int(round(_bounce(o["x0"], o["vx"], t, W - o["w"])))
        y = int(round(_bounce(o["y0"], o["vy"], t, H - o["h"])))
        return x, y

    def frame(self, t: int):
        cfg = self.cfg
        H, W = cfg.H, cfg.W
        rgb = self.bg_rgb.copy()
        depth = self.bg_depth.copy()
        gt = np.zeros((H, W), np.bool_)
        objmask = np.zeros((H, W), np.bool_)
        placed = []
        if self.camo is not None:
            x, y = self._pos(self.camo, t)
            sl = (slice(y, y + self.camo["h"]), slice(x, x + self.camo["w"]))
            depth[sl] -= float(cfg.camouflage_offset_mm)
            gt[sl] = True
        for o in self.objects:
            x, y = self._pos(o, t)
            placed.append((o, x, y))
            objmask[y:y + o["h"], x:x + o["w"]] = True
        if cfg.shadows:
            for o, x, y in placed:
                sx, sy = x + int(round(0.15 * o["w"])), y + int(round(0.10 * o["h"]))
                sl = (slice(sy, min(H, sy + o["h"])), slice(sx, min(W, sx + o["w"])))
                sub = rgb[sl]
                keep = ~objmask[sl]
                sub[keep] = np.rint(np.float32(0.6) * sub[keep])
        for o, x, y in placed:
            rgb[y:y + o["h"], x:x + o["w"]] = o["rgb"]
            depth[y:y + o["h"], x:x + o["w"]] = float(cfg.near_mm)
            gt[y:y + o["h"], x:x + o["w"]] = True
        if cfg.illumination:
            rgb += np.float32(_triangle(t))

        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg.seed, 1, t])))
        if cfg.rgb_noise > 0:
            rgb += np.rint(rng.standard_normal((H, W, 3), dtype=np.float32) * np.float32(cfg.rgb_noise))
        if cfg.depth_noise_mm > 0:
            depth += np.rint(rng.standard_normal((H, W), dtype=np.float32) * np.float32(cfg.depth_noise_mm))
        rgb8 = np.clip(rgb, 0.0, 255.0).astype(np.uint8)
        d16 = np.clip(depth, 1.0, 65535.0).astype(np.uint16)
        if cfg.hole_frac > 0:
            d16[rng.random((H, W), dtype=np.float32) < np.float32(cfg.hole_frac)] = 0
        return rgb8, d16, (gt.astype(np.uint8) * np.uint8(255))

    def frames(self, t0: int, n: int):
        """Frames t0 .. t0+n-1 stacked: rgb [n,H,W,3], depth [n,H,W], gt [n,H,W]."""
        out = [self.frame(t) for t in range(t0, t0 + n)]
        return (np.stack([o[0] for o in out]), np.stack([o[1] for o in out]),
                np.stack([o[2] for o in out]))
