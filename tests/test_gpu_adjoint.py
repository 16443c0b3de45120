"""GPU adjoint of the GMM window against the fp64 reference (oracle/adjoint.py).

Bar: the forward (Z, term flags, recorded choices) identical to the oracle's fp32 recording
forward; dL/dtheta within 1e-3 relative of the fp64 reverse sweep (itself pinned against
central finite differences); the same gradient for every checkpoint interval; Adam on theta
lowers the loss of the 640x480, 64-frame workload."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log  # noqa: E402
from oracle.adjoint import bce_loss_and_grad, fd_gradient, record_window, replay_window, reverse_gradient  # noqa: E402
from oracle.gmm import GmmParams  # noqa: E402
from synth import Scene, preset  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _params_c(p: GmmParams):
    from paper_2002_00250_amd import fgs
    c = fgs.fgs_gmm_params_default()
    c.Kc, c.Kd = p.Kc, p.Kd
    c.alpha, c.lambda_, c.T_bg, c.w_init = p.alpha, p.lam, p.T_bg, p.w_init
    c.v_init_c, c.v_min_c, c.v_init_d, c.v_min_d = p.v_init_c, p.v_min_c, p.v_init_d, p.v_min_d
    c.w_depth, c.depth_max_mm = p.w_depth, p.depth_max_mm
    return c


def _dev(rgb, dep, gt=None):
    r = torch.from_numpy(np.ascontiguousarray(rgb)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(dep).view(np.int16)).cuda()
    return (r, d) if gt is None else (r, d, torch.from_numpy(np.ascontiguousarray(gt)).cuda())


def _decode(rec, K, shift):
    r = (rec >> np.uint64(shift)).astype(np.uint64) & np.uint64(0xFFFFFFFF)
    r = r.astype(np.int64)
    term = (r & 1) != 0
    argmin = (r >> 1) & 7
    active = (r >> 4) & 1
    ks = (r >> 5) & 7
    clamp = (r >> 8) & 1
    perm = np.stack([(r >> (9 + 3 * k)) & 7 for k in range(K)], axis=1)
    return term, argmin, active.astype(bool), np.where(ks == 7, -1, ks), clamp.astype(bool), perm


@pytest.mark.parametrize("K,H,W,T", [(3, 48, 64, 40), (5, 21, 37, 33), (1, 8, 8, 20)])
def test_window_forward_and_records_match_oracle(K, H, W, T):
    from paper_2002_00250_amd.adjoint import GmmWindow
    p = GmmParams(Kc=K, Kd=K)
    rgb, dep, _ = Scene(preset("adjoint_640x480", H=H, W=W)).frames(0, T)
    Z, has, dc, dd = record_window(rgb, dep, p)
    win = GmmWindow(T, H, W, _params_c(p), checkpoint_every=16)
    theta = torch.tensor([p.alpha, p.lam, p.w_depth], dtype=torch.float32, device="cuda")
    Zg, hg = win.forward(theta, *_dev(rgb, dep))
    torch.cuda.synchronize()
    nz = int((Zg.cpu().numpy() != Z).sum())
    log(f"window forward K={K} {H}x{W}x{T}: Z differs at {nz} of {Z.size}")
    assert nz == 0
    np.testing.assert_array_equal(hg.cpu().numpy().astype(bool), has)
    rec = win.records()
    for dec, sh in ((dc, 0), (dd, 32)):
        term, argmin, active, ks, clamp, perm = _decode(rec, K, sh)
        np.testing.assert_array_equal(term, dec.term)
        np.testing.assert_array_equal(active, dec.active)
        np.testing.assert_array_equal(ks, dec.kstar)
        np.testing.assert_array_equal(clamp, dec.clamp)
        np.testing.assert_array_equal(np.where(dec.term, argmin, 0), np.where(dec.term, dec.argmin, 0))
        np.testing.assert_array_equal(np.where(active[:, None], perm, 0), np.where(dec.active[:, None], dec.perm, 0))
    win.close()


def _oracle_grad(rgb, dep, gt, p, theta):
    Z, has, dc, dd = record_window(rgb, dep, p, theta)
    Z64 = replay_window(rgb, dep, p, dc, dd, theta, np.float64)
    loss, dZ = bce_loss_and_grad(Z64, has, gt)
    return loss, dZ, reverse_gradient(rgb, dep, p, dc, dd, theta, dZ), (has, dc, dd)


@pytest.mark.parametrize("E", [16, 5, 64])
def test_window_gradient_end_to_end_matches_fp64_reference(E):
    from paper_2002_00250_amd.adjoint import GmmWindow, GmmWindowFunction, window_bce_loss
    p = GmmParams(Kc=3, Kd=3)
    H, W, T = 40, 56, 64
    rgb, dep, gt = Scene(preset("adjoint_640x480", H=H, W=W)).frames(0, T)
    theta0 = (0.01, 2.5, 1.0)
    loss_ref, dZ, g_ref, (has, dc, dd) = _oracle_grad(rgb, dep, gt, p, theta0)
    win = GmmWindow(T, H, W, _params_c(p), checkpoint_every=E)
    theta = torch.tensor(theta0, dtype=torch.float32, device="cuda", requires_grad=True)
    r, d, g = _dev(rgb, dep, gt)
    Z, hasg = GmmWindowFunction.apply(theta, r, d, win)
    loss = window_bce_loss(Z, hasg, g)
    loss.backward()
    gg = theta.grad.double().cpu().numpy()
    rel = np.abs(gg - g_ref) / np.abs(g_ref)
    log(f"adjoint {H}x{W}x{T} E={E}: loss gpu {loss.item():.6f} ref {loss_ref:.6f}; grad gpu {gg} ref {g_ref} rel {rel}")
    assert abs(loss.item() - loss_ref) <= 1e-4 * abs(loss_ref)
    assert np.all(rel <= 1e-3)
    if E == 16:
        fd = fd_gradient(rgb, dep, gt, p, dc, dd, has, theta0)
        rel_fd = np.abs(gg - fd) / np.abs(fd)
        log(f"adjoint vs central differences (fp64, choices frozen): fd {fd} rel {rel_fd}")
        assert np.all(rel_fd <= 1e-3)
    win.close()


def test_two_applications_on_one_window():
    # Two forwards on one window before the backward (two thetas in one loss): each
    # gradient is that of its own forward, against the fp64 reference at its theta.
    from paper_2002_00250_amd.adjoint import GmmWindow, GmmWindowFunction, window_bce_loss
    p = GmmParams(Kc=3, Kd=3)
    H, W, T = 24, 40, 40
    rgb, dep, gt = Scene(preset("adjoint_640x480", H=H, W=W)).frames(0, T)
    thetas = [(0.01, 2.5, 1.0), (0.03, 2.0, 0.5)]
    refs = [_oracle_grad(rgb, dep, gt, p, th)[2] for th in thetas]
    win = GmmWindow(T, H, W, _params_c(p), checkpoint_every=16)
    r, d, g = _dev(rgb, dep, gt)
    ts = [torch.tensor(th, dtype=torch.float32, device="cuda", requires_grad=True) for th in thetas]
    losses = [window_bce_loss(*GmmWindowFunction.apply(t, r, d, win), g) for t in ts]
    assert win.forwards == 2
    (losses[0] + losses[1]).backward()
    for t, g_ref, th in zip(ts, refs, thetas):
        gg = t.grad.double().cpu().numpy()
        rel = np.abs(gg - g_ref) / np.abs(g_ref)
        log(f"two applications on one window, theta {th}: grad gpu {gg} ref {g_ref} rel {rel}")
        assert np.all(rel <= 1e-3)
    # backward of the first application alone, after the second one's forward
    ts = [torch.tensor(th, dtype=torch.float32, device="cuda", requires_grad=True) for th in thetas]
    first = window_bce_loss(*GmmWindowFunction.apply(ts[0], r, d, win), g)
    window_bce_loss(*GmmWindowFunction.apply(ts[1], r, d, win), g)
    first.backward()
    rel = np.abs(ts[0].grad.double().cpu().numpy() - refs[0]) / np.abs(refs[0])
    assert np.all(rel <= 1e-3), rel
    win.close()


def test_window_gradient_through_the_variance_floor():
    # a fast rate puts the variances on their floors inside the window: the clamped steps'
    # adjoints must vanish on the GPU as in the fp64 reference
    from paper_2002_00250_amd.adjoint import GmmWindow, GmmWindowFunction, window_bce_loss
    p = GmmParams(Kc=3, Kd=3)
    H, W, T = 40, 56, 48
    rgb, dep, gt = Scene(preset("adjoint_640x480", H=H, W=W)).frames(0, T)
    theta0 = (0.15, 2.5, 1.0)
    loss_ref, dZ, g_ref, (has, dc, dd) = _oracle_grad(rgb, dep, gt, p, theta0)
    assert dc.clamp.sum() >= 10 and dd.clamp.sum() >= 10
    win = GmmWindow(T, H, W, _params_c(p), checkpoint_every=16)
    theta = torch.tensor(theta0, dtype=torch.float32, device="cuda", requires_grad=True)
    r, d, g = _dev(rgb, dep, gt)
    Z, hasg = GmmWindowFunction.apply(theta, r, d, win)
    loss = window_bce_loss(Z, hasg, g)
    loss.backward()
    gg = theta.grad.double().cpu().numpy()
    rel = np.abs(gg - g_ref) / np.abs(g_ref)
    log(f"adjoint alpha=0.15 ({int(dc.clamp.sum())} + {int(dd.clamp.sum())} clamped steps): grad gpu {gg} "
        f"ref {g_ref} rel {rel}")
    assert abs(loss.item() - loss_ref) <= 1e-4 * abs(loss_ref)
    assert np.all(rel <= 1e-3)
    win.close()


def test_window_gradient_640x480_64_frames_sampled_pixels():
    # The 640x480, K=3, 64-frame, checkpoint-16 workload at full size.  Each pixel's
    # recursion is independent, so feeding dL/dZ on a sample of pixels (zero elsewhere)
    # makes the GPU gradient the sum over that sample, which the oracle computes exactly.
    from paper_2002_00250_amd.adjoint import GmmWindow
    p = GmmParams(Kc=3, Kd=3)
    H, W, T = 480, 640, 64
    rgb, dep, gt = Scene(preset("adjoint_640x480")).frames(0, T)
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(H * W, 3000, replace=False))
    ys, xs = sel // W, sel % W
    theta0 = (0.01, 2.5, 1.0)
    s_rgb, s_dep, s_gt = rgb[:, ys, xs][:, None], dep[:, ys, xs][:, None], gt[:, ys, xs][:, None]
    _, dZs, g_ref, _ = _oracle_grad(s_rgb, s_dep, s_gt, p, theta0)
    dZ = np.zeros((T, H, W), np.float32)
    dZ[:, ys, xs] = dZs[:, 0].astype(np.float32)
    win = GmmWindow(T, H, W, _params_c(p), checkpoint_every=16)
    theta = torch.tensor(theta0, dtype=torch.float32, device="cuda")
    r, d = _dev(rgb, dep)
    Z, has = win.forward(theta, r, d)
    gg = win.backward(theta, r, d, torch.from_numpy(dZ).cuda()).cpu().numpy()
    rel = np.abs(gg - g_ref) / np.abs(g_ref)
    log(f"adjoint 640x480x64 on {sel.size} sampled px: grad gpu {gg} ref {g_ref} rel {rel}")
    assert np.all(rel <= 1e-3)
    win.close()


def test_adam_on_theta_lowers_the_loss():
    from paper_2002_00250_amd.adjoint import GmmWindow, GmmWindowFunction, window_bce_loss
    p = GmmParams(Kc=3, Kd=3)
    H, W, T = 480, 640, 64
    rgb, dep, gt = Scene(preset("adjoint_640x480")).frames(0, T)
    r, d, g = _dev(rgb, dep, gt)
    win = GmmWindow(T, H, W, _params_c(p), checkpoint_every=16)
    theta = torch.tensor([0.01, 2.5, 1.0], dtype=torch.float32, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([{"params": [theta]}], lr=1e-2)
    scale = torch.tensor([1e-2, 1.0, 1.0], device="cuda")   # per-parameter step size
    lo = torch.tensor([1e-4, 0.5, 0.0], device="cuda")
    hi = torch.tensor([0.5, 10.0, 10.0], device="cuda")
    losses = []
    for step in range(200):
        opt.zero_grad()
        Z, has = GmmWindowFunction.apply(theta, r, d, win)
        loss = window_bce_loss(Z, has, g)
        loss.backward()
        theta.grad.mul_(scale)
        opt.step()
        with torch.no_grad():
            theta.copy_(torch.maximum(torch.minimum(theta, hi), lo))
        losses.append(loss.item())
    log(f"adam 640x480x64, 200 steps: loss {losses[0]:.4f} -> {losses[-1]:.4f} (min {min(losses):.4f}); "
        f"theta {theta.detach().cpu().numpy()}")
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.9 * losses[0]
    win.close()
