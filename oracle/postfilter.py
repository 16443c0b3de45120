"""Median post-filter of a binary foreground mask.  Oracle (test infrastructure only).

The paper's method leaves its masks unfiltered (Sec. 3); the base PBAS method it builds
on smooths its output mask with a median filter.  Definition used here: every pixel is
background (0) or foreground (any nonzero value, read as 255); output pixel (y, x) is the
median, the middle value in sorted order, of the (2r+1) x (2r+1) window centred on it,
where window pixels beyond the image repeat the nearest edge pixel.
"""
from __future__ import annotations

import numpy as np


def median_mask(mask, radius: int, rows: slice | None = None) -> np.ndarray:
    """The median-filtered mask (uint8, 0/255) by the definition above: sort each window
    and take its middle element.  `rows` restricts the output to a band of rows (the
    window still reads the whole image)."""
    m = np.where(np.asarray(mask) != 0, 255, 0).astype(np.uint8)
    if m.ndim != 2:
        raise ValueError("mask must be 2-D")
    H, W = m.shape
    r = int(radius)
    if r < 0:
        raise ValueError("radius must be >= 0")
    y0, y1, _ = (rows or slice(0, H)).indices(H)
    if H == 0 or W == 0 or y1 <= y0:
        return np.zeros((max(0, y1 - y0), W), np.uint8)
    k = 2 * r + 1
    padded = np.pad(m, r, mode="edge")          # replicated border
    out = np.empty((y1 - y0, W), np.uint8)
    for a in range(y0, y1, 32):                 # bands of output rows bound the memory
        b = min(y1, a + 32)
        win = np.lib.stride_tricks.sliding_window_view(padded[a:b + 2 * r], (k, k))
        flat = win.reshape(b - a, W, k * k)
        out[a - y0:b - y0] = np.sort(flat, axis=-1)[..., (k * k) // 2]
    return out
