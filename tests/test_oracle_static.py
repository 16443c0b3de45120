"""Pins for the static-object oracle (reading R-24 of Sec. 6's future-work item): hand-derived
masks (tests/golden), the window definition (static iff the last M masks are all foreground)
computed directly on random sequences, M = 1, and the 16-bit saturation of the run counter."""
import json
import os

import numpy as np

from oracle.static import COUNTER_MAX, StaticRef

GOLD = os.path.join(os.path.dirname(__file__), "golden", "static_hand_cases.json")


def test_hand_derived_sequence():
    g = json.load(open(GOLD))
    ref = StaticRef(1, 3, g["M"])
    for m, exp in zip(g["masks"], g["static"]):
        got = ref.step(np.array([m], np.uint8))
        assert got[0].tolist() == exp, g["note"]


def test_window_definition_on_random_masks():
    rng = np.random.default_rng(4)
    for M in (1, 2, 5, 11):
        T, H, W = 60, 9, 13
        p = rng.uniform(0.5, 0.97, (H, W))
        masks = (rng.random((T, H, W)) < p).astype(np.uint8) * rng.integers(1, 256, (T, H, W)).astype(np.uint8)
        ref = StaticRef(H, W, M)
        for t in range(T):
            got = ref.step(masks[t]) != 0
            if t + 1 < M:
                exp = np.zeros((H, W), bool)
            else:
                exp = (masks[t + 1 - M:t + 1] != 0).all(axis=0)
            np.testing.assert_array_equal(got, exp, err_msg=f"M={M} t={t}")


def test_m_one_is_the_mask():
    rng = np.random.default_rng(1)
    ref = StaticRef(4, 5, 1)
    for _ in range(10):
        m = rng.integers(0, 2, (4, 5)).astype(np.uint8) * 255
        np.testing.assert_array_equal(ref.step(m), m)


def test_counter_saturates_at_16_bits():
    ref = StaticRef(1, 2, COUNTER_MAX)
    ref.count[:] = COUNTER_MAX - 2
    fg = np.array([[255, 255]], np.uint8)
    assert ref.step(fg).tolist() == [[0, 0]]             # count 65534 < M
    assert ref.step(fg).tolist() == [[255, 255]]         # 65535 = M
    assert ref.step(fg).tolist() == [[255, 255]]         # stays at 65535
    assert ref.count.tolist() == [[COUNTER_MAX, COUNTER_MAX]]
    assert ref.step(np.array([[255, 0]], np.uint8)).tolist() == [[255, 0]]
    assert ref.count.tolist() == [[COUNTER_MAX, 0]]
