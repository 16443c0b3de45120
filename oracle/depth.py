"""Depth conversion to the 8-bit code both background models work on.

Oracle (test infrastructure only).

Sec. 4.2 converts the sensor's uint16 depth map to 8 bits so that depth can
be modelled like a colour channel, quoting an accuracy of about 4 cm over the
sensor's 0.1-10 m range (Sec. 4.1).  Taken literally, 0..65535 -> 0..255 would
give 257 mm steps, which contradicts the 4 cm figure; a 10 m full scale gives
10000/255 = 39.2 mm per level, which matches it.  Reading used here:

    q(D) = 0                                        if D == 0 (invalid)
    q(D) = min(255, max(1, floor((255*D + M//2) / M)))   otherwise

with full scale M = ``depth_max_mm`` (default 10000 mm): round-half-up
integer rescaling, with the code 0 reserved for "no depth" (Sec. 3.1 and 3.2
use depth only where the sensor value is greater than 0).

Parity: pinned by the values the reading fixes (900 -> 23, 1500 -> 38,
3000 -> 77), by the 39.2 mm step, and by monotonicity; see
``tests/test_oracle_depth.py``.
"""
from __future__ import annotations

import numpy as np

DEPTH_MAX_MM = 10000


def depth_q8(depth, depth_max_mm: int = DEPTH_MAX_MM) -> np.ndarray:
    """uint16 depth in mm -> uint8 depth code (0 = invalid), as defined above (R-03,
    from Sec. 4.2's 16-to-8-bit conversion)."""
    d = np.asarray(depth).astype(np.int64)
    m = int(depth_max_mm)
    q = (255 * d + m // 2) // m
    q = np.minimum(255, np.maximum(1, q))
    return np.where(d == 0, 0, q).astype(np.uint8)


def depth_valid(depth) -> np.ndarray:
    """Depth is used only where the sensor reports a value greater than 0 (Sec. 3.1, 3.2)."""
    return np.asarray(depth) > 0


def upscale_nearest(depth, H: int, W: int) -> np.ndarray:
    """Depth map brought to an H x W grid by nearest neighbour on pixel centres (Sec. 4.3:
    depth is upscaled to the RGB resolution when they differ):
    out[y, x] = depth[floor((y + 1/2) Hd / H), floor((x + 1/2) Wd / W)]."""
    d = np.asarray(depth)
    Hd, Wd = d.shape
    ys = ((2 * np.arange(H, dtype=np.int64) + 1) * Hd) // (2 * H)
    xs = ((2 * np.arange(W, dtype=np.int64) + 1) * Wd) // (2 * W)
    return d[ys][:, xs]
