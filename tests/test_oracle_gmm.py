"""Pins for the GMM oracle (Sec. 3.1 and the Stauffer-Grimson mixture it adapts).

Each test checks the oracle against something other than itself: closed forms of the
recursion under a constant input, hand-derived cases (tests/golden), the textbook
colour-only Stauffer-Grimson rule that the RGB-D decision must reduce to, and
invariants of the model."""
import json
import os

import numpy as np
import pytest

from oracle.gmm import GmmParams, GmmRef
from oracle.depth import depth_q8
from synth import Scene, preset

GOLD = os.path.join(os.path.dirname(__file__), "golden", "gmm_hand_cases.json")


def _params(**kw):
    return GmmParams(**kw)


def _single(params, wc, muc, vc, wd=None, mud=None, vd=None, dtype=np.float32):
    """A 1x1 model with a given state."""
    g = GmmRef(1, 1, params, dtype=dtype)
    Kc, Kd = params.Kc, params.Kd
    st = dict(w_c=np.array(wc, dtype).reshape(Kc, 1, 1),
              mu_c=np.array(muc, dtype).reshape(Kc, 3, 1, 1),
              v_c=np.array(vc, dtype).reshape(Kc, 1, 1),
              w_d=np.array(wd if wd is not None else [0] * Kd, dtype).reshape(Kd, 1, 1),
              mu_d=np.array(mud if mud is not None else [0] * Kd, dtype).reshape(Kd, 1, 1),
              v_d=np.array(vd if vd is not None else [params.v_init_d] * Kd, dtype).reshape(Kd, 1, 1),
              t=5)
    g.set_state_planes(st)
    return g


def _frame(rgb, D):
    return (np.array(rgb, np.uint8).reshape(1, 1, 3), np.array([[D]], np.uint16))


def test_hand_replacement_and_match_cases():
    gold = json.load(open(GOLD))
    p = _params(**gold["params"])
    for case in gold["replacement_cases"]:
        g = _single(p, case["w"], case["mu"], case["v"])
        m = g.step(*_frame(case["X"], 0))
        st = g.state_planes()
        np.testing.assert_allclose(st["w_c"][:, 0, 0], case["expect_w"], rtol=2e-6, atol=1e-7,
                                   err_msg=case["name"])
        np.testing.assert_allclose(st["mu_c"][:, :, 0, 0], case["expect_mu"], rtol=2e-6,
                                   err_msg=case["name"])
        np.testing.assert_allclose(st["v_c"][:, 0, 0], case["expect_v"], rtol=2e-6, err_msg=case["name"])
        assert np.isclose(g.last_Z[0, 0], case["expect_Z"], rtol=1e-6), case["name"]
        assert m[0, 0] == case["expect_mask"], case["name"]


def test_hand_decision_cases():
    gold = json.load(open(GOLD))
    dc = gold["decision_cases"][0]
    for c in dc["cases"]:
        p = _params(**{**gold["params"], "w_depth": c["w_depth"]})
        g = _single(p, [1, 0, 0], [[100, 100, 100], [0, 0, 0], [0, 0, 0]], [3, 675, 675],
                    wd=[1, 0, 0], mud=[40, 0, 0], vd=[1, 25, 25])
        m = g.step(*_frame(dc["rgb"], c["D"]))
        assert g.last_Z[0, 0] == np.float32(c["Z"]), c
        assert m[0, 0] == c["mask"], c


def test_constant_frame_from_fresh_model_closed_form():
    # Fresh model, constant input X: frame 0 seeds (w_init, X, v_init) -> w = 1; afterwards
    # mu_t = X exactly, w_0 = 1 exactly, v_t = max(v_min, (1-alpha)^t v_init), mask 0.
    p = _params(Kc=3, Kd=3)
    H, W = 2, 3
    rng = np.random.default_rng(0)
    rgb = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    D = rng.integers(200, 9000, (H, W)).astype(np.uint16)
    g = GmmRef(H, W, p)
    a = 1.0 - float(np.float32(p.alpha))
    for t in range(520):
        m = g.step(rgb, D)
        assert not m.any()
        st = g.state_planes()
        n = t  # updates after the seeding frame
        assert np.all(st["w_c"][0] == 1) and np.all(st["w_c"][1:] == 0)
        assert np.all(st["w_d"][0] == 1) and np.all(st["w_d"][1:] == 0)
        np.testing.assert_array_equal(st["mu_c"][0], np.moveaxis(rgb, -1, 0).astype(np.float32))
        np.testing.assert_array_equal(st["mu_d"][0], depth_q8(D).astype(np.float32))
        vc = max(p.v_min_c, a ** n * p.v_init_c)
        vd = max(p.v_min_d, a ** n * p.v_init_d)
        np.testing.assert_allclose(st["v_c"][0], vc, rtol=1e-4)
        np.testing.assert_allclose(st["v_d"][0], vd, rtol=1e-4)
    # the floors bind after ln(v_min/v_init)/ln(a) frames (about 401 colour, 320 depth)
    assert np.all(g.state_planes()["v_c"][0] == np.float32(p.v_min_c))
    assert np.all(g.state_planes()["v_d"][0] == np.float32(p.v_min_d))


def test_constant_frame_from_offset_mean_closed_form():
    # Gaussian 0 starts at mu_0 = X + Delta_0 within lambda sigma; others far and weak.
    # Closed forms (a = 1 - alpha): mu_t - X = a^t Delta_0,
    # v_t = a^t (v_0 + |Delta_0|^2 a (1 - a^t)), w_t = 1 - a^t (1 - w_0).
    p = _params(Kc=3, Kd=1)
    X = np.array([120.0, 80.0, 60.0])
    deltas = np.array([[3.0, -2.0, 1.0], [0.5, 0.5, 0.5], [-6.0, 4.0, 2.0], [0.0, 0.0, 7.0]])
    v0, w0 = 400.0, 0.6
    n = len(deltas)
    g = GmmRef(1, n, p)
    st = g.state_planes()
    st = dict(st)
    st["w_c"] = np.array([[[w0] * n], [[0.3] * n], [[0.1] * n]], np.float32)
    mu = np.zeros((3, 3, 1, n), np.float32)
    for i in range(n):
        mu[0, :, 0, i] = X + deltas[i]
        mu[1, :, 0, i] = [250, 250, 250]
        mu[2, :, 0, i] = [0, 250, 0]
    st["mu_c"] = mu
    st["v_c"] = np.array([[[v0] * n], [[100.0] * n], [[100.0] * n]], np.float32)
    g.set_state_planes(st)
    rgb = np.broadcast_to(X.astype(np.uint8), (1, n, 3)).copy()
    D = np.zeros((1, n), np.uint16)
    a = 1.0 - float(np.float32(p.alpha))
    for t in range(1, 200):
        g.step(rgb, D)
        s = g.state_planes()
        at = a ** t
        exp_mu = X[None, :] + at * deltas
        np.testing.assert_allclose(s["mu_c"][0, :, 0, :].T, exp_mu, rtol=1e-4, atol=1e-4)
        d2 = (deltas ** 2).sum(1)
        exp_v = at * (v0 + d2 * a * (1 - at))
        np.testing.assert_allclose(s["v_c"][0, 0], exp_v, rtol=1e-4)
        np.testing.assert_allclose(s["w_c"][0, 0], 1 - at * (1 - w0), rtol=1e-5)
        np.testing.assert_allclose(s["w_c"][1, 0], at * 0.3, rtol=1e-4)


def _stauffer_grimson_rgb(state, rgb, p):
    """The textbook colour-only test and update, written in its own form (float64):
    background = leading Gaussians whose weights first exceed T; the pixel is background
    iff it lies within lambda sigma of one of them.  Update:
    w <- (1-alpha) w + alpha M;  mu <- (1-rho) mu + rho X;  s2 <- (1-rho) s2 + rho |X-mu|^2."""
    w, mu, v = state["w_c"].astype(np.float64), state["mu_c"].astype(np.float64), state["v_c"].astype(np.float64)
    K, H, W = w.shape
    X = np.moveaxis(rgb.astype(np.float64), -1, 0)
    fg = np.zeros((H, W), bool)
    nw, nmu, nv = w.copy(), mu.copy(), v.copy()
    lam, al = float(p.lam), float(np.float32(p.alpha))
    for y in range(H):
        for x in range(W):
            ww, mm, vv = w[:, y, x], mu[:, :, y, x], v[:, y, x]
            if ww[0] > 0:
                csum, B = 0.0, int((ww > 0).sum())
                for k in range(K):
                    csum += ww[k]
                    if csum > p.T_bg:
                        B = k + 1
                        break
                dist2 = ((X[:, y, x][None] - mm) ** 2).sum(1)
                fg[y, x] = not any(dist2[k] < lam * lam * vv[k] for k in range(B))
            match = [k for k in range(K) if ww[k] > 0 and ((X[:, y, x] - mm[k]) ** 2).sum() < lam * lam * vv[k]]
            Mv = np.zeros(K)
            if match:
                k = match[0]
                Mv[k] = 1
                newmu = (1 - al) * mm[k] + al * X[:, y, x]
                s2 = (1 - al) * vv[k] + al * ((X[:, y, x] - newmu) ** 2).sum()
                nmu[k, :, y, x] = newmu
                nv[k, y, x] = max(s2, p.v_min_c)
                nw_ = (1 - al) * ww + al * Mv
            else:
                nw_ = (1 - al) * ww
                nw_[K - 1] = p.w_init
                nmu[K - 1, :, y, x] = X[:, y, x]
                nv[K - 1, y, x] = p.v_init_c
            nw_ = nw_ / nw_.sum()
            keys = nw_ / np.sqrt(nv[:, y, x])
            order = sorted(range(K), key=lambda k: -keys[k])
            nw[:, y, x] = nw_[order]
            nmu[:, :, y, x] = nmu[order, :, y, x]
            nv[:, y, x] = nv[order, y, x]
    return fg, nw, nmu, nv


@pytest.mark.parametrize("mode", ["no_depth", "zero_depth_weight"])
def test_reduces_to_stauffer_grimson_without_depth(mode):
    p = _params(Kc=3, Kd=3, w_depth=0.0 if mode == "zero_depth_weight" else 1.0)
    sc = Scene(preset("gmm_320x240", H=12, W=16, n_objects=2))
    g = GmmRef(12, 16, p, dtype=np.float64)
    for t in range(40):
        rgb, D, _ = sc.frame(t)
        if mode == "no_depth":
            D = np.zeros_like(D)
        before = {k: v.copy() if isinstance(v, np.ndarray) else v for k, v in g.state_planes().items()}
        m = g.step(rgb, D)
        fg, nw, nmu, nv = _stauffer_grimson_rgb(before, rgb, p)
        if t > 0:
            np.testing.assert_array_equal(m == 255, fg, err_msg=f"frame {t}")
        s = g.state_planes()
        # the two algebraic forms round differently; a formula slip would show at O(alpha)
        np.testing.assert_allclose(s["w_c"], nw, rtol=1e-7, atol=1e-10)
        np.testing.assert_allclose(s["mu_c"], nmu, rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(s["v_c"], nv, rtol=1e-7)


def test_invariants_on_moving_scene():
    p = _params(Kc=5, Kd=5)
    sc = Scene(preset("hd_1280x720", H=48, W=64))
    g = GmmRef(48, 64, p)
    for t in range(60):
        rgb, D, _ = sc.frame(t)
        g.step(rgb, D)
        s = g.state_planes()
        for w, v, vmin in ((s["w_c"], s["v_c"], p.v_min_c), (s["w_d"], s["v_d"], p.v_min_d)):
            used = w[0] > 0
            assert np.all(np.abs(w.sum(0)[used] - 1) <= 1e-6)
            assert np.all(v >= np.float32(vmin))
            assert np.all(w >= 0)
            key = w / np.sqrt(v)
            assert np.all(np.diff(key, axis=0) <= 0)      # ranked by w/sigma, descending
        assert np.all(s["w_c"][0] > 0)                      # colour model always has data


def test_static_noise_free_scene_gives_empty_mask():
    cfg = preset("gmm_320x240", H=24, W=32, n_objects=0, rgb_noise=0.0, depth_noise_mm=0.0,
                 hole_frac=0.0)
    sc = Scene(cfg)
    g = GmmRef(24, 32, _params())
    for t in range(30):
        rgb, D, _ = sc.frame(t)
        assert not g.step(rgb, D).any()


def test_colour_camouflage_needs_depth():
    # An object whose colour equals the background but 600 mm nearer: foreground only
    # when the depth model takes part (the case Sec. 5 reports as the biggest gain).
    H, W = 20, 20
    rng = np.random.default_rng(5)
    bg = rng.integers(60, 200, (H, W, 3)).astype(np.uint8)
    D = np.full((H, W), 2000, np.uint16)
    obj = np.zeros((H, W), bool)
    obj[5:12, 6:14] = True
    res = {}
    for use_depth in (True, False):
        g = GmmRef(H, W, _params())
        for t in range(40):
            g.step(bg, D if use_depth else np.zeros_like(D))
        D2 = D.copy()
        D2[obj] = 1400
        m = g.step(bg, D2 if use_depth else np.zeros_like(D2))
        res[use_depth] = m
    assert np.all(res[True][obj] == 255) and not res[True][~obj].any()
    assert not res[False].any()


def test_invalid_depth_leaves_depth_model_untouched():
    g = GmmRef(4, 4, _params())
    sc = Scene(preset("gmm_320x240", H=4, W=4, n_objects=0))
    for t in range(5):
        g.step(*sc.frame(t)[:2])
    before = {k: np.array(v, copy=True) for k, v in g.state_planes().items() if k != "t"}
    rgb, D, _ = sc.frame(5)
    D[1, 2] = 0
    g.step(rgb, D)
    after = g.state_planes()
    for k in ("w_d", "mu_d", "v_d"):
        np.testing.assert_array_equal(after[k][:, 1, 2], before[k][:, 1, 2])
    assert not np.array_equal(after["v_d"][:, 0, 0], before["v_d"][:, 0, 0])  # valid: updated


def _scalar_step(state, rgb, D, p):
    """Brute force: one pixel at a time in Python float32 scalars, following the same
    definitions.  Used on tiny images only."""
    f = np.float32
    a, al, lam2 = f(1) - f(p.alpha), f(p.alpha), f(p.lam) * f(p.lam)
    Kc, H, W = state["w_c"].shape
    out = {k: np.array(v, copy=True) for k, v in state.items() if k != "t"}
    mask = np.zeros((H, W), np.uint8)
    q8 = depth_q8(D)
    for y in range(H):
        for x in range(W):
            models = [("c", [f(v) for v in rgb[y, x]], True, f(p.w_init), f(p.v_init_c), f(p.v_min_c)),
                      ("d", [f(q8[y, x])], D[y, x] > 0, f(p.w_init), f(p.v_init_d), f(p.v_min_d))]
            terms = []
            for name, X, active, wi, vi, vmin in models:
                w = [f(v) for v in out["w_" + name][:, y, x]]
                mu = ([[f(c) for c in out["mu_c"][k, :, y, x]] for k in range(Kc)] if name == "c"
                      else [[f(out["mu_d"][k, y, x])] for k in range(len(w))])
                v = [f(s) for s in out["v_" + name][:, y, x]]
                K = len(w)
                q = []
                for k in range(K):
                    d2 = f(0)
                    for c in range(len(X)):
                        e = f(X[c] - mu[k][c])
                        d2 = f(e * e) if c == 0 else f(d2 + f(e * e))
                    q.append(f(d2 / v[k]))
                if w[0] > 0 and active:
                    cum, B = f(0), sum(1 for s in w if s > 0)
                    for k in range(K):
                        cum = f(cum + w[k])
                        if cum > f(p.T_bg):
                            B = k + 1
                            break
                    terms.append((name, min(q[:B])))
                if not active:
                    continue
                ks = next((k for k in range(K) if w[k] > 0 and q[k] < lam2), None)
                w = [f(a * s) for s in w]
                if ks is not None:
                    w[ks] = f(w[ks] + al)
                    mu[ks] = [f(m + f(al * f(X[c] - m))) for c, m in enumerate(mu[ks])]
                    d2 = f(0)
                    for c in range(len(X)):
                        e = f(X[c] - mu[ks][c])
                        d2 = f(e * e) if c == 0 else f(d2 + f(e * e))
                    v[ks] = max(f(v[ks] + f(al * f(d2 - v[ks]))), vmin)
                else:
                    w[K - 1], mu[K - 1], v[K - 1] = wi, list(X), vi
                S = w[0]
                for k in range(1, K):
                    S = f(S + w[k])
                w = [f(s / S) for s in w]
                keys = [f(w[k] / np.sqrt(v[k])) for k in range(K)]
                order = sorted(range(K), key=lambda k: -keys[k])   # Python's sort is stable
                out["w_" + name][:, y, x] = [w[k] for k in order]
                out["v_" + name][:, y, x] = [v[k] for k in order]
                if name == "c":
                    out["mu_c"][:, :, y, x] = [mu[k] for k in order]
                else:
                    out["mu_d"][:, y, x] = [mu[k][0] for k in order]
            Z = None
            for name, delta in terms:
                tterm = f(delta - lam2) if name == "c" else f(f(p.w_depth) * f(delta - lam2))
                Z = tterm if Z is None else f(Z + tterm)
            mask[y, x] = 255 if (Z is not None and Z >= 0) else 0
    return mask, out


def test_vectorised_equals_scalar_brute_force():
    p = _params(Kc=3, Kd=2)
    sc = Scene(preset("gmm_320x240", H=5, W=6, n_objects=1))
    g = GmmRef(5, 6, p)
    for t in range(25):
        rgb, D, _ = sc.frame(t)
        st = {k: np.array(v, copy=True) if k != "t" else v for k, v in g.state_planes().items()}
        m = g.step(rgb, D)
        m2, out = _scalar_step(st, rgb, D, p)
        np.testing.assert_array_equal(m, m2)
        s = g.state_planes()
        for k in out:
            np.testing.assert_array_equal(s[k], out[k], err_msg=f"{k} frame {t}")


@pytest.mark.parametrize("rho_mode", [1, 0])
def test_rho_over_w_makes_mean_the_weighted_sample_mean(rho_mode):
    # With rho = alpha / w (w the matched weight after its update) and weights that sum
    # to 1, w*mu of every Gaussian obeys m_t = (1 - alpha) m_{t-1} + alpha X_t [matched],
    # like w_t = (1 - alpha) w_{t-1} + alpha [matched]; so mu_t = m_t / w_t is the
    # exponentially weighted mean of the samples the Gaussian was matched with.  Two far
    # clusters, samples within +-2 of their centre (always matched by their own Gaussian),
    # fp64.  With rho = alpha the identity must fail.
    alpha = 0.05
    p = _params(Kc=2, Kd=1, alpha=alpha, rho_mode=rho_mode)
    n, T = 6, 80
    A = np.array([50.0, 60.0, 70.0])
    B = np.array([200.0, 190.0, 180.0])
    g = GmmRef(1, n, p, dtype=np.float64)
    st = dict(g.state_planes())
    st["w_c"] = np.array([[[0.75] * n], [[0.25] * n]])
    mu = np.zeros((2, 3, 1, n))
    mu[0, :, 0, :] = A[:, None]
    mu[1, :, 0, :] = B[:, None]
    st["mu_c"] = mu
    st["v_c"] = np.full((2, 1, n), 400.0)
    g.set_state_planes(st)
    rng = np.random.default_rng(3)
    wA, wB = np.full(n, 0.75), np.full(n, 0.25)
    mA, mB = wA[:, None] * A, wB[:, None] * B
    worst = 0.0
    for t in range(T):
        pickA = rng.random(n) < 0.6
        X = np.where(pickA[:, None], A, B) + rng.integers(-2, 3, size=(n, 3))
        g.step(X.astype(np.uint8).reshape(1, n, 3), np.zeros((1, n), np.uint16))
        wA = (1 - alpha) * wA + alpha * pickA
        wB = (1 - alpha) * wB + alpha * ~pickA
        mA = (1 - alpha) * mA + alpha * X * pickA[:, None]
        mB = (1 - alpha) * mB + alpha * X * ~pickA[:, None]
        s = g.state_planes()
        muc = s["mu_c"][:, :, 0, :]                     # [K, 3, n]
        slotA = np.argmin(np.abs(muc[:, 0, :] - A[0]), axis=0)
        for i in range(n):
            a_, b_ = slotA[i], 1 - slotA[i]
            np.testing.assert_allclose(s["w_c"][a_, 0, i], wA[i], rtol=1e-12)
            np.testing.assert_allclose(s["w_c"][b_, 0, i], wB[i], rtol=1e-12)
            worst = max(worst, np.abs(muc[a_, :, i] - mA[i] / wA[i]).max(),
                        np.abs(muc[b_, :, i] - mB[i] / wB[i]).max())
    if rho_mode == 1:
        assert worst < 1e-9
    else:
        assert worst > 0.05


def _row_model(p, n, wc, muc, vc, wd, mud, vd, dtype=np.float32):
    """A 1 x n model whose pixels all hold the same mixtures."""
    g = GmmRef(1, n, p, dtype=dtype)
    Kc, Kd = p.Kc, p.Kd
    rep = lambda a, *shape: np.broadcast_to(np.array(a, dtype).reshape(*shape, 1, 1), shape + (1, n)).copy()
    g.set_state_planes(dict(w_c=rep(wc, Kc), mu_c=rep(muc, Kc, 3), v_c=rep(vc, Kc),
                            w_d=rep(wd, Kd), mu_d=rep(mud, Kd), v_d=rep(vd, Kd), t=5))
    return g


def test_density_decision_closed_form_at_the_mean():
    # X on the mean of the only colour Gaussian, no depth: P = s / (2 pi v) (Eq. (1) at d = 0).
    s_ = 10000.0
    for v0 in (12.0, 27.5, 400.0, 675.0):
        p = _params(Kc=3, Kd=1, decision=1, density_scale=s_)
        X = [37, 140, 201]
        g = _row_model(p, 1, [1, 0, 0], [X, [0, 0, 0], [0, 0, 0]], [v0, 675, 675], [0], [0], [25])
        g.step(np.array(X, np.uint8).reshape(1, 1, 3), np.zeros((1, 1), np.uint16))
        np.testing.assert_allclose(float(g.last_P[0, 0]), s_ / (2 * np.pi * v0), rtol=2e-6)


@pytest.mark.parametrize("with_depth", [True, False])
def test_density_decision_agrees_with_log_sum_rule(with_depth):
    # One Gaussian per model, equal variances everywhere.  With tau = s^2 e^{-lam^2} /
    # (4 pi^2 v_c v_d) (colour only: s e^{-lam^2/2} / (2 pi v_c)), "P < tau" is
    # "delta_c + delta_d > 2 lam^2" (colour only: "delta_c > lam^2"): the log-sum rule
    # (R-09, w_d = 1) must give the same masks except on the boundary itself.
    rng = np.random.default_rng(7)
    n, s_, lam = 4000, 10000.0, 2.5
    Vc, Vd = 60.0, 4.0
    mu_c, mu_code = np.array([120.0, 90.0, 60.0]), 100
    tau = (s_ ** 2 * np.exp(-lam ** 2) / (4 * np.pi ** 2 * Vc * Vd)) if with_depth else \
        (s_ * np.exp(-lam ** 2 / 2) / (2 * np.pi * Vc))
    kw = dict(Kc=1, Kd=1, lam=lam, w_depth=1.0)
    X = np.clip(mu_c + rng.normal(0, 14, size=(n, 3)), 0, 255).round().astype(np.uint8)
    codes = np.clip(mu_code + rng.integers(-6, 7, size=n), 1, 255)
    mm = np.round(codes * 10000 / 255).astype(np.uint16) if with_depth else np.zeros(n, np.uint16)
    masks = []
    for dec in (0, 1):
        p = _params(decision=dec, density_scale=s_, density_threshold=float(tau), **kw)
        g = _row_model(p, n, [1], [mu_c], [Vc], [1], [mu_code], [Vd], dtype=np.float64)
        masks.append(g.step(X.reshape(1, n, 3), mm.reshape(1, n))[0])
    dc = ((X - mu_c) ** 2).sum(1) / Vc
    dd = (depth_q8(mm, 10000).astype(float) - mu_code) ** 2 / Vd if with_depth else 0.0
    margin = np.abs(dc + dd - (2 if with_depth else 1) * lam ** 2)
    differ = masks[0] != masks[1]
    assert masks[0].any() and not masks[0].all()
    assert not differ[margin > 1e-6].any()


def test_density_decision_uses_the_gaussian_attaining_delta():
    # Two background Gaussians (weights 0.5, 0.4 > T_bg together); X on the mean of the
    # second: delta = 0 is attained by Gaussian 1, so P = s / (2 pi v_1), not v_0.
    p = _params(Kc=3, Kd=1, decision=1, T_bg=0.7)
    X = [200, 30, 90]
    g = _row_model(p, 1, [0.5, 0.4, 0.1], [[10, 10, 10], X, [250, 0, 0]], [100.0, 33.0, 500.0],
                   [0], [0], [25])
    g.step(np.array(X, np.uint8).reshape(1, 1, 3), np.zeros((1, 1), np.uint16))
    np.testing.assert_allclose(float(g.last_P[0, 0]), 10000.0 / (2 * np.pi * 33.0), rtol=2e-6)


def test_rho_alpha_eta_closed_form_on_a_constant_scene():
    # Stauffer-Grimson's rate rho = alpha * eta(X | mu, v) with eta = exp(-q/2) / (2 pi v)
    # (Eq. (1)).  A constant frame on the mean of the only colour Gaussian keeps q = 0, so
    # rho_t = alpha / (2 pi v_t) and the variance follows v_{t+1} = v_t (1 - alpha / (2 pi v_t))
    # = v_t - alpha / (2 pi): it falls by exactly alpha/(2 pi) per frame until the floor
    # (rho = alpha would give v_t = (1 - alpha)^t v_0 instead).
    alpha, v0 = 0.05, 30.0
    p = _params(Kc=3, Kd=1, alpha=alpha, rho_mode=2, v_min_c=12.0)
    X = [77, 88, 99]
    g = _row_model(p, 1, [1, 0, 0], [X, [0, 0, 0], [0, 0, 0]], [v0, 675, 675], [0], [0], [25],
                   dtype=np.float64)
    rgb = np.array(X, np.uint8).reshape(1, 1, 3)
    for t in range(1, 60):
        g.step(rgb, np.zeros((1, 1), np.uint16))
        v = float(g.state_planes()["v_c"][0, 0, 0])
        np.testing.assert_allclose(v, max(v0 - t * alpha / (2 * np.pi), 12.0), rtol=1e-12)


def test_per_channel_variances_reduce_to_isotropic_on_grey_input():
    # Grey input (R = G = B) keeps every mean grey and every channel deviation equal, so a
    # per-channel model whose variances start at v_init/3 and whose threshold is 3 lambda^2
    # is the isotropic model in other units: q_diag = 3 q_iso, v_c = v_iso / 3 per channel,
    # identical weights, means, ranking and masks (no depth; fp64).
    rng = np.random.default_rng(11)
    H, W, T = 6, 40, 50
    lam = 2.5
    iso = GmmRef(H, W, _params(Kc=3, Kd=1, lam=lam), dtype=np.float64)
    dia = GmmRef(H, W, _params(Kc=3, Kd=1, lam=lam * np.sqrt(3.0), var_mode=1), dtype=np.float64)
    base = rng.integers(40, 200, size=(H, W))
    for t in range(T):
        g = np.clip(base + rng.integers(-4, 5, size=(H, W)) + (60 if 20 <= t < 28 else 0), 0, 255)
        g[:, : 8 + t % 5] = 255 - g[:, : 8 + t % 5]          # a moving grey object
        rgb = np.repeat(g.astype(np.uint8)[..., None], 3, axis=-1)
        D = np.zeros((H, W), np.uint16)
        assert np.array_equal(iso.step(rgb, D), dia.step(rgb, D)), t
        a, b = iso.state_planes(), dia.state_planes()
        np.testing.assert_allclose(b["w_c"], a["w_c"], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(b["mu_c"], a["mu_c"], rtol=1e-12)
        for c in range(3):
            np.testing.assert_allclose(b["v_c"][:, c], a["v_c"] / 3.0, rtol=1e-12)


def test_per_channel_variances_decay_independently():
    # A constant frame on the mean of the only colour Gaussian: each channel's variance
    # decays as (1 - alpha)^t from its own start and is floored at v_min/3 on its own.
    alpha, vmin = 0.05, 12.0
    p = _params(Kc=2, Kd=1, alpha=alpha, v_min_c=vmin, var_mode=1)
    X = [50, 150, 250]
    v0 = np.array([300.0, 40.0, 4.5])
    g = GmmRef(1, 1, p, dtype=np.float64)
    st = dict(g.state_planes())
    st["w_c"] = np.array([1.0, 0.0]).reshape(2, 1, 1)
    st["mu_c"] = np.array([X, [0, 0, 0]], float).reshape(2, 3, 1, 1)
    st["v_c"] = np.array([v0, [225.0] * 3]).reshape(2, 3, 1, 1)
    g.set_state_planes(st)
    for t in range(1, 80):
        g.step(np.array(X, np.uint8).reshape(1, 1, 3), np.zeros((1, 1), np.uint16))
        v = g.state_planes()["v_c"][0, :, 0, 0]
        np.testing.assert_allclose(v, np.maximum((1 - alpha) ** t * v0, vmin / 3), rtol=1e-9)
