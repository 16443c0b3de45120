"""Pins for the fp64 adjoint reference (oracle/adjoint.py): its recording forward is the GMM
oracle step for step; its hand-written reverse sweep agrees with central finite differences
of the replayed loss; its loss and dL/dZ agree with torch's BCE-with-logits."""
import numpy as np
import pytest

from oracle.adjoint import (bce_loss_and_grad, fd_gradient, record_window, replay_window,
                            reverse_gradient)
from oracle.gmm import GmmParams, GmmRef
from synth import Scene, preset


def _frames(H, W, T, **kw):
    return Scene(preset("adjoint_640x480", H=H, W=W, **kw)).frames(0, T)


@pytest.mark.parametrize("K", [2, 3, 5])
def test_recording_forward_is_the_gmm_oracle(K):
    p = GmmParams(Kc=K, Kd=K)
    rgb, dep, _ = _frames(12, 17, 30)
    Z, has, dc, dd = record_window(rgb, dep, p)
    g = GmmRef(12, 17, p)
    for t in range(30):
        g.step(rgb[t], dep[t])
        np.testing.assert_array_equal(np.where(g.last_has_term, g.last_Z, 0), Z[t])
        np.testing.assert_array_equal(g.last_has_term, has[t])
    # replaying the recorded choices in fp32 at the recorded theta reproduces Z exactly
    np.testing.assert_array_equal(replay_window(rgb, dep, p, dc, dd, (p.alpha, p.lam, p.w_depth), np.float32), Z)


@pytest.mark.parametrize("K,theta", [(3, (0.01, 2.5, 1.0)), (3, (0.03, 2.0, 0.4)), (5, (0.01, 2.5, 1.0))])
def test_reverse_sweep_matches_central_differences(K, theta):
    p = GmmParams(Kc=K, Kd=K)
    rgb, dep, gt = _frames(16, 20, 48)
    Z, has, dc, dd = record_window(rgb, dep, p, theta)
    Z64 = replay_window(rgb, dep, p, dc, dd, theta, np.float64)
    _, dZ = bce_loss_and_grad(Z64, has, gt)
    g = reverse_gradient(rgb, dep, p, dc, dd, theta, dZ)
    fd = fd_gradient(rgb, dep, gt, p, dc, dd, has, theta)
    assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(fd) + 1e-9), (g, fd)
    assert abs(g[0]) > 0 and abs(g[1]) > 0 and abs(g[2]) > 0


def test_no_depth_means_no_depth_weight_gradient():
    p = GmmParams(Kc=3, Kd=3)
    rgb, dep, gt = _frames(10, 12, 20)
    dep = np.zeros_like(dep)
    theta = (p.alpha, p.lam, p.w_depth)
    Z, has, dc, dd = record_window(rgb, dep, p)
    _, dZ = bce_loss_and_grad(replay_window(rgb, dep, p, dc, dd, theta), has, gt)
    g = reverse_gradient(rgb, dep, p, dc, dd, theta, dZ)
    assert g[2] == 0.0
    # dZ/dlambda = -2 lambda wherever the colour term exists
    assert np.isclose(g[1], float((dZ * (-2 * p.lam) * dc.term).sum()), rtol=1e-12)


def test_loss_matches_torch_bce_with_logits():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    Z = rng.normal(0, 30, (5, 6, 7))
    has = rng.random((5, 6, 7)) < 0.8
    gt = np.where(rng.random((5, 6, 7)) < 0.3, 255, 0)
    loss, g = bce_loss_and_grad(Z, has, gt, t0=1, tau=2.0)
    Zt = torch.tensor(Z, dtype=torch.float64, requires_grad=True)
    w = torch.tensor(has[1:], dtype=torch.float64)
    y = torch.tensor(gt[1:] != 0, dtype=torch.float64)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(Zt[1:] / 2.0, y, weight=w, reduction="sum") / w.sum()
    lt.backward()
    assert np.isclose(loss, lt.item(), rtol=1e-12)
    np.testing.assert_allclose(g, Zt.grad.numpy(), rtol=1e-10, atol=1e-15)
