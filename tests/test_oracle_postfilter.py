"""Pins of the median post-filter oracle: hand-worked masks, the library median filter
with a replicated border, a count over explicitly clamped coordinates on small images,
and the filter's symmetries."""
import json
import os

import numpy as np
import pytest

from oracle.postfilter import median_mask

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "median_hand_cases.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def test_hand_cases():
    for c in _cases():
        got = median_mask(np.array(c["mask"], np.uint8), c["radius"])
        assert np.array_equal(got, np.array(c["expected"], np.uint8)), c["name"]


@pytest.mark.parametrize("H,W,r,p", [(1, 1, 3, 0.5), (6, 9, 1, 0.5), (23, 41, 2, 0.4), (40, 37, 4, 0.6),
                                     (50, 60, 7, 0.5), (2, 70, 5, 0.5), (70, 3, 6, 0.3)])
def test_matches_library_median(H, W, r, p):
    # scipy's median filter with mode "nearest" repeats the edge pixel beyond the border
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(H * 1000 + W * 10 + r)
    m = np.where(rng.random((H, W)) < p, 255, 0).astype(np.uint8)
    assert np.array_equal(median_mask(m, r), ndimage.median_filter(m, size=2 * r + 1, mode="nearest"))


@pytest.mark.parametrize("r", [0, 1, 2, 3])
def test_majority_over_clamped_coordinates(r):
    # brute force on a small image: count foreground over the window with every coordinate
    # clamped into the image, and compare with half the window
    rng = np.random.default_rng(r)
    H, W = 7, 9
    m = rng.integers(0, 3, (H, W)).astype(np.uint8) * rng.integers(0, 200, (H, W)).astype(np.uint8)
    n = (2 * r + 1) ** 2
    exp = np.zeros((H, W), np.uint8)
    for y in range(H):
        for x in range(W):
            cnt = 0
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    yy, xx = min(max(y + dy, 0), H - 1), min(max(x + dx, 0), W - 1)
                    cnt += int(m[yy, xx] != 0)
            exp[y, x] = 255 if 2 * cnt > n else 0
    assert np.array_equal(median_mask(m, r), exp)


def test_symmetries():
    rng = np.random.default_rng(11)
    m = np.where(rng.random((31, 45)) < 0.5, 255, 0).astype(np.uint8)
    for r in (1, 3, 6):
        f = median_mask(m, r)
        assert np.array_equal(median_mask(m.T, r), f.T)                 # transpose
        assert np.array_equal(median_mask(m[:, ::-1], r), f[:, ::-1])   # mirror
        assert np.array_equal(median_mask(255 - m, r), 255 - f)         # complement (odd window)
    for r in (0, 2, 7):
        assert not median_mask(np.zeros((5, 8), np.uint8), r).any()
        assert (median_mask(np.full((5, 8), 9, np.uint8), r) == 255).all()


def test_row_band_and_empty():
    rng = np.random.default_rng(5)
    m = np.where(rng.random((90, 33)) < 0.5, 255, 0).astype(np.uint8)
    full = median_mask(m, 3)
    assert np.array_equal(median_mask(m, 3, rows=slice(40, 77)), full[40:77])
    assert median_mask(np.zeros((0, 5), np.uint8), 2).shape == (0, 5)
    assert median_mask(np.zeros((4, 0), np.uint8), 2).shape == (4, 0)
