"""Static-object detection on a sequence of foreground masks.

Oracle (test infrastructure only).

The paper names the detection of static objects as future work (Sec. 6) and gives no
method.  Reading used here: a pixel belongs to a static object when the segmenter has
marked it foreground in each of the last M frames.  Per pixel, a run counter

    c_t = min(c_{t-1} + 1, 65535)   if mask_t != 0
    c_t = 0                          otherwise                 (c before the first frame: 0)

and the static mask static_t = 255 where c_t >= M, else 0 (M >= 1).  The counter
saturates at 65535 (it is kept in 16 bits); static pixels stay static while they stay
foreground.  The detector only reads the masks: it does not feed back into the
background model.
"""
from __future__ import annotations

import numpy as np

COUNTER_MAX = 65535


class StaticRef:
    """Run counters over H x W masks; ``step(mask) -> static mask`` (uint8 0/255)."""

    def __init__(self, H: int, W: int, M: int):
        if M < 1:
            raise ValueError("M must be >= 1")
        self.M = M
        self.count = np.zeros((H, W), np.int64)

    def step(self, mask: np.ndarray) -> np.ndarray:
        fg = np.asarray(mask) != 0
        self.count = np.where(fg, np.minimum(self.count + 1, COUNTER_MAX), 0)
        return np.where(self.count >= self.M, 255, 0).astype(np.uint8)
