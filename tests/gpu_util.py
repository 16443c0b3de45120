"""Helpers for the GPU tests: device upload of synthetic frames and parity accounting."""
from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(rgb: np.ndarray, depth: np.ndarray):
    import torch
    r = torch.from_numpy(np.ascontiguousarray(rgb)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(depth).view(np.int16)).cuda()
    return r, d


def rel_close(a, b, rtol=1e-4, atol=1e-7):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) <= rtol * np.maximum(np.abs(a), np.abs(b)) + atol


def compare_gmm_state(gpu: dict, ref: dict, rtol=1e-4):
    """Return (n_values, n_bad, n_not_bitequal) over all GMM planes."""
    n = bad = neq = 0
    for k in ("w_c", "mu_c", "v_c", "w_d", "mu_d", "v_d"):
        g = np.asarray(gpu[k], np.float32)
        r = np.asarray(ref[k], np.float32)
        assert g.shape == r.shape, (k, g.shape, r.shape)
        n += g.size
        bad += int((~rel_close(g, r, rtol)).sum())
        neq += int((g.view(np.uint32) != r.view(np.uint32)).sum())
    return n, bad, neq


def compare_pbas_state(gpu: dict, ref: dict, rtol=1e-4):
    """Integer state must be exact; R, T within rtol.  Returns a dict of mismatch counts."""
    out = {}
    for k in ("samples", "dhist", "S"):
        out[k] = int((np.asarray(gpu[k]) != np.asarray(ref[k])).sum())
    for k in ("R", "T"):
        g = np.asarray(gpu[k], np.float32)
        r = np.asarray(ref[k], np.float32)
        out[k] = int((~rel_close(g, r, rtol)).sum())
        out[k + "_bits"] = int((g.view(np.uint32) != r.view(np.uint32)).sum())
    return out


def compare_pbas_grad_state(gpu: dict, ref: dict, rtol=1e-4):
    """The gradient-magnitude variant: sample words and magnitudes and the magnitude sums
    exact; D, S, R, T within rtol (and counted where not bit-equal)."""
    out = {}
    for k in ("samples", "gsamples", "gsum"):
        out[k] = int((np.asarray(gpu[k]) != np.asarray(ref[k])).sum())
    for k in ("dhist", "S", "R", "T"):
        g = np.asarray(gpu[k], np.float32)
        r = np.asarray(ref[k], np.float32)
        assert g.shape == r.shape, (k, g.shape, r.shape)
        out[k] = int((~rel_close(g, r, rtol)).sum())
        out[k + "_bits"] = int((g.view(np.uint32) != r.view(np.uint32)).sum())
    return out
