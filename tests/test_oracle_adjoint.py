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


def test_reverse_sweep_through_the_variance_floor():
    # a fast rate drives both variances onto their floors inside the window, so the clamped
    # steps (whose variance no longer depends on theta) are part of what is differentiated
    p = GmmParams(Kc=3, Kd=3)
    theta = (0.15, 2.5, 1.0)
    rgb, dep, gt = _frames(16, 20, 48)
    Z, has, dc, dd = record_window(rgb, dep, p, theta)
    assert dc.clamp.sum() >= 10 and dd.clamp.sum() >= 10
    Z64 = replay_window(rgb, dep, p, dc, dd, theta, np.float64)
    _, dZ = bce_loss_and_grad(Z64, has, gt)
    g = reverse_gradient(rgb, dep, p, dc, dd, theta, dZ)
    fd = fd_gradient(rgb, dep, gt, p, dc, dd, has, theta)
    assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(fd) + 1e-9), (g, fd)


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


def test_lambda_and_depth_weight_gradients_in_closed_form():
    # with the choices frozen, Z is affine in w_d with slope delta_d - lambda^2 where the depth
    # term exists (0 elsewhere), and dZ/dlambda = -2 lambda (term_c + w_d term_d): the sweep's
    # lambda and w_d gradients are dL/dZ summed against these per pixel
    p = GmmParams(Kc=3, Kd=3)
    rgb, dep, gt = _frames(14, 18, 24)
    theta = (p.alpha, p.lam, 0.7)
    Z, has, dc, dd = record_window(rgb, dep, p, theta)
    assert dd.term.any() and (dc.term & ~dd.term).any()
    Z64 = replay_window(rgb, dep, p, dc, dd, theta)
    _, dZ = bce_loss_and_grad(Z64, has, gt)
    g = reverse_gradient(rgb, dep, p, dc, dd, theta, dZ)
    slope = (replay_window(rgb, dep, p, dc, dd, (theta[0], theta[1], 1.0)) -
             replay_window(rgb, dep, p, dc, dd, (theta[0], theta[1], 0.0)))
    assert np.all(slope[~dd.term] == 0) and np.any(slope[dd.term] != 0)
    assert np.isclose(g[2], float((dZ * slope).sum()), rtol=1e-10)
    dZ_dlam = -2.0 * theta[1] * (dc.term + theta[2] * dd.term)
    assert np.isclose(g[1], float((dZ * dZ_dlam).sum()), rtol=1e-10)


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


def _torch_replay_Z(torch, rgb, dep, p, dc, dd, theta):
    """Z_t(theta) written afresh in float64 torch ops from the update rules (recorded choices
    held fixed): matched mean and variance update with the variance floor where it was
    applied, replacement of the last rank, the recorded ranking, and the score on the
    pre-update models."""
    from oracle.depth import depth_q8
    T, H, W = dep.shape
    alpha, lam, wd = theta
    f64 = torch.float64

    def step(mu, v, X, dec, t, v_init, v_min):
        K = mu.shape[0]
        ks = torch.as_tensor(dec.kstar[t])
        act = torch.as_tensor(dec.active[t])
        clamp = torch.as_tensor(dec.clamp[t])
        mus, vs = [], []
        for k in range(K):
            hit = act & (ks == k)
            m_new = mu[k] + alpha * (X - mu[k])
            v_new = v[k] + alpha * (((X - m_new) ** 2).sum(0) - v[k])
            v_new = torch.where(clamp, torch.full_like(v_new, v_min), v_new)
            mus.append(torch.where(hit[None], m_new, mu[k]))
            vs.append(torch.where(hit, v_new, v[k]))
        rep = act & (ks < 0)
        mus[K - 1] = torch.where(rep[None], X, mus[K - 1])
        vs[K - 1] = torch.where(rep, torch.full_like(vs[K - 1], v_init), vs[K - 1])
        mu_n, v_n = torch.stack(mus), torch.stack(vs)
        perm = torch.as_tensor(dec.perm[t])
        mu_s = torch.gather(mu_n, 0, perm[:, None].expand_as(mu_n))
        v_s = torch.gather(v_n, 0, perm)
        return torch.where(act[None, None], mu_s, mu), torch.where(act[None], v_s, v)

    def delta(mu, v, X, a):
        a = torch.as_tensor(a)
        m = torch.gather(mu, 0, a[None, None].expand(1, mu.shape[1], *a.shape))[0]
        vv = torch.gather(v, 0, a[None])[0]
        return ((X - m) ** 2).sum(0) / vv

    muc = torch.zeros((p.Kc, 3, H, W), dtype=f64)
    vc = torch.full((p.Kc, H, W), p.v_init_c, dtype=f64)
    mud = torch.zeros((p.Kd, 1, H, W), dtype=f64)
    vd = torch.full((p.Kd, H, W), p.v_init_d, dtype=f64)
    Zs = []
    for t in range(T):
        Xc = torch.as_tensor(np.moveaxis(rgb[t], -1, 0).astype(np.float64))
        Xd = torch.as_tensor(depth_q8(dep[t], p.depth_max_mm).astype(np.float64))[None]
        tc = delta(muc, vc, Xc, dc.argmin[t]) - lam * lam
        td = wd * (delta(mud, vd, Xd, dd.argmin[t]) - lam * lam)
        on_c, on_d = torch.as_tensor(dc.term[t]), torch.as_tensor(dd.term[t])
        zero = torch.zeros_like(tc)
        Zs.append(torch.where(on_c, torch.where(on_d, tc + td, tc), torch.where(on_d, td, zero)))
        muc, vc = step(muc, vc, Xc, dc, t, p.v_init_c, p.v_min_c)
        mud, vd = step(mud, vd, Xd, dd, t, p.v_init_d, p.v_min_d)
    return torch.stack(Zs)


@pytest.mark.parametrize("theta", [(0.01, 2.5, 1.0), (0.05, 1.8, 0.6)])
def test_reverse_sweep_matches_torch_autograd_on_32x32(theta):
    # the hand-written reverse sweep against torch.autograd (float64) through an independent
    # torch replay of the same window, 32 x 32 crop, K = 3
    torch = pytest.importorskip("torch")
    p = GmmParams(Kc=3, Kd=3)
    rgb, dep, gt = _frames(32, 32, 24, n_objects=2)
    Z, has, dc, dd = record_window(rgb, dep, p, theta)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    Zt = _torch_replay_Z(torch, rgb, dep, p, dc, dd, (th[0], th[1], th[2]))
    Z64 = replay_window(rgb, dep, p, dc, dd, theta, np.float64)
    np.testing.assert_allclose(Zt.detach().numpy(), Z64, rtol=1e-12, atol=1e-9)
    w = torch.tensor(has[1:], dtype=torch.float64)
    y = torch.tensor(gt[1:] != 0, dtype=torch.float64)
    loss = torch.nn.functional.binary_cross_entropy_with_logits(Zt[1:], y, weight=w, reduction="sum") / w.sum()
    loss.backward()
    _, dZ = bce_loss_and_grad(Z64, has, gt)
    g = reverse_gradient(rgb, dep, p, dc, dd, theta, dZ)
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-9, atol=1e-12)
    assert np.all(np.abs(g) > 0)
