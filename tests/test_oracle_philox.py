"""Pins for the oracle's Philox4x32-10 (Salmon et al., SC'11): the ROCm random-number
library's implementation of the same bijection, compiled for the host, must give the
same words; plus the two oracle implementations against each other and basic statistics."""
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10, philox4x32_10_int


def _cases(n, seed=11):
    rng = np.random.default_rng(seed)
    c = rng.integers(0, 2**32, size=(n, 6), dtype=np.uint64)
    fixed = np.array([[0] * 6, [2**32 - 1] * 6, [1, 2, 3, 4, 5, 6], [7, 0, 1, 0, 0x2002, 0x250]],
                     np.uint64)
    return np.concatenate([fixed, c])


def test_matches_rocm_library(rocrand_probe):
    cases = _cases(3000)
    text = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([rocrand_probe], input=text, capture_output=True, text=True, check=True)
    lib = np.array([[int(v) for v in line.split()] for line in out.stdout.strip().splitlines()],
                   np.uint64)
    assert lib.shape == (len(cases), 4)
    ours = np.stack(philox4x32_10(cases[:, 0], cases[:, 1], cases[:, 2], cases[:, 3], 0, 0), -1)
    # numpy version takes one key per call: evaluate row by row for per-row keys
    for i in range(len(cases)):
        k0, k1 = int(cases[i, 4]), int(cases[i, 5])
        v = philox4x32_10(cases[i, 0], cases[i, 1], cases[i, 2], cases[i, 3], k0, k1)
        ours[i] = [int(x) for x in v]
        if i < 200:
            assert philox4x32_10_int(cases[i, :4], (k0, k1)) == tuple(int(x) for x in lib[i])
    np.testing.assert_array_equal(ours.astype(np.uint64), lib)


def test_vectorised_equals_integer_version():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2**32, size=(500, 4), dtype=np.uint64)
    k = (0x12345678, 0x9ABCDEF0)
    v = np.stack(philox4x32_10(c[:, 0], c[:, 1], c[:, 2], c[:, 3], *k), -1)
    for i in range(len(c)):
        assert tuple(int(x) for x in v[i]) == philox4x32_10_int(c[i], k)


def test_uniformity_and_avalanche():
    n = 1 << 16
    v = np.stack(philox4x32_10(np.arange(n, dtype=np.uint64), 5, 0, 0, 99, 0), -1)
    top = (v >> np.uint32(28)).ravel()
    counts = np.bincount(top, minlength=16)
    exp = top.size / 16
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 45.0                    # 15 dof, p ~ 1e-4
    # flipping one counter bit flips about half of the 128 output bits
    a = np.stack(philox4x32_10(np.arange(4096, dtype=np.uint64), 0, 0, 0, 1, 2), -1)
    b = np.stack(philox4x32_10(np.arange(4096, dtype=np.uint64) ^ np.uint64(1 << 17), 0, 0, 0, 1, 2), -1)
    flips = np.unpackbits((a ^ b).view(np.uint8)).reshape(4096, 128).sum(1)
    assert abs(flips.mean() - 64) < 1.0
