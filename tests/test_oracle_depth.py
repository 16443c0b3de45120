"""Pins for the depth code (Sec. 4.1-4.2): 0 = no depth, ~39.2 mm per level at 10 m
full scale, round-half-up integer rescaling."""
from fractions import Fraction

import numpy as np

from oracle.depth import depth_q8, depth_valid


def test_values_fixed_by_reading():
    d = np.array([0, 1, 900, 1500, 2400, 3000, 10000, 65535], np.uint16)
    assert depth_q8(d).tolist() == [0, 1, 23, 38, 61, 77, 255, 255]


def test_exact_rational_rescaling():
    # floor(255*D/10000 + 1/2) in exact rational arithmetic, clamped to [1, 255].
    rng = np.random.default_rng(7)
    ds = np.concatenate([np.arange(1, 3000), rng.integers(1, 65536, 5000)]).astype(np.uint16)
    got = depth_q8(ds)
    for D, g in zip(ds.tolist(), got.tolist()):
        q = int(Fraction(255 * D, 10000) + Fraction(1, 2))  # int() floors a positive Fraction
        assert g == min(255, max(1, q)), D


def test_step_is_about_4cm_and_monotone():
    d = np.arange(1, 10001, dtype=np.uint16)
    q = depth_q8(d).astype(np.int64)
    assert np.all(np.diff(q) >= 0)
    edges = np.nonzero(np.diff(q))[0]
    step = np.diff(edges).mean()
    assert abs(step - 10000 / 255) < 0.5       # 39.2 mm per code (about 4 cm)
    assert q.min() == 1 and q.max() == 255


def test_validity_is_depth_positive():
    assert depth_valid(np.array([0, 1, 65535], np.uint16)).tolist() == [False, True, True]


def test_other_full_scale():
    # A 65535 mm full scale puts 257 mm in one code (the literal 16-bit -> 8-bit rescale).
    q = depth_q8(np.array([128, 129, 385, 386, 65535], np.uint16), depth_max_mm=65535)
    assert q.tolist() == [1, 1, 1, 2, 255]


def test_upscale_nearest_identity_and_integer_factor():
    from oracle.depth import upscale_nearest
    rng = np.random.default_rng(1)
    d = rng.integers(0, 5000, (6, 9)).astype(np.uint16)
    np.testing.assert_array_equal(upscale_nearest(d, 6, 9), d)
    up = upscale_nearest(d, 12, 18)            # factor 2: every sample becomes a 2x2 block
    np.testing.assert_array_equal(up, np.repeat(np.repeat(d, 2, 0), 2, 1))


def test_upscale_nearest_centres_for_480_to_720():
    from oracle.depth import upscale_nearest
    d = np.arange(480, dtype=np.uint16)[:, None] * np.ones((1, 3), np.uint16)
    up = upscale_nearest(d, 720, 3)
    # output row y samples input row floor((y + 1/2) * 480 / 720): 0,1,1,2,3,3,...
    assert up[:8, 0].tolist() == [0, 1, 1, 2, 3, 3, 4, 5]
    assert up[-1, 0] == 479
    counts = np.bincount(up[:, 0], minlength=480)
    assert set(counts.tolist()) == {1, 2} and counts.sum() == 720
