"""Adjoint of the RGB-D GMM recursion over a window of frames (reference, fp64).

Oracle (test infrastructure only).

Parameters theta = (alpha, lambda, w_d): learning rate, match threshold in standard
deviations and depth weight of the RGB-D GMM (Sec. 3.1 and the readings in
``oracle.gmm``).  The window starts from a fresh model at frame 0 and yields the
pre-update score Z_t of every frame (Z = (delta_c - lambda^2) + w_d (delta_d - lambda^2),
terms only where the model has data and, for depth, D > 0).

Decisions frozen.  The recursion has discrete choices: the background set B, the
Gaussian that attains delta (first index of the minimum over k < B), the matched
Gaussian k* or the replacement, the variance floor, and the ranking permutation.
``record_window`` runs the recursion in fp32 exactly as ``oracle.gmm.GmmRef`` does and
records those choices.  ``replay_window`` recomputes everything continuous with the
choices held fixed, in any precision and for any theta, so the loss becomes a smooth
function of theta whose gradient is what the adjoint computes.

With the choices fixed, the weights reach Z only through B, k* and the ranking, i.e. not
at all continuously; their adjoints vanish and the gradient with respect to alpha flows
through the matched Gaussian's mean and variance updates:

    mu'  = mu + alpha (X - mu)                 d mu'/d mu = (1 - alpha),  d mu'/d alpha = X - mu
    v~   = v + alpha (|X - mu'|^2 - v)         d v~/d v = (1 - alpha),    d v~/d mu' = -2 alpha (X - mu')
                                               d v~/d alpha = |X - mu'|^2 - v
    v'   = v_min if the floor applied, else v~
    delta = |X - mu_a|^2 / v_a                 d/d mu_a = -2 (X - mu_a) / v_a,  d/d v_a = -delta / v_a
    Z: dZ/d delta_c = 1, dZ/d delta_d = w_d, dZ/d lambda = -2 lambda (1 + w_d [depth term]),
       dZ/d w_d = delta_d - lambda^2 [depth term]

A replaced Gaussian takes constants (adjoint zero); an unmatched, unreplaced Gaussian's
mean and variance pass through; an inactive depth model passes its state through.

``reverse_gradient`` is the hand-written reverse sweep; ``fd_gradient`` the central finite
difference of the replayed loss (decisions frozen), used to check it.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .depth import depth_q8
from .gmm import GmmParams, background_count, first_match, fresh_mixture, sq_distances


@dataclass
class Decisions:
    """The discrete choices of the Sec. 3.1 step (R-08..R-12), recorded to be held fixed.
    Per frame and model: term [T,H,W] bool, argmin a [T,H,W], active [T,H,W],
    kstar [T,H,W] (-1 = replaced), clamp [T,H,W], perm [T,K,H,W] (old index per new rank)."""
    term: np.ndarray
    argmin: np.ndarray
    active: np.ndarray
    kstar: np.ndarray
    clamp: np.ndarray
    perm: np.ndarray


def _first_argmin(q: np.ndarray, B: np.ndarray):
    """delta = min_{k<B} q_k with the first index attaining it (sequential strict '<')."""
    delta = q[0].copy()
    a = np.zeros(q.shape[1:], np.int64)
    for k in range(1, q.shape[0]):
        take = (k < B) & (q[k] < delta)
        delta = np.where(take, q[k], delta)
        a = np.where(take, k, a)
    return delta, a


def _record_model_step(mix, X, active, alpha, lam2, T_bg, w_init, v_init, v_min):
    """One fp32 step of one mixture, as oracle.gmm.update_mixture, recording the choices."""
    f = mix.w.dtype.type
    K, C = mix.mu.shape[0], mix.mu.shape[1]
    q = sq_distances(mix, X) / mix.v
    used = mix.w[0] > 0
    delta, a = _first_argmin(q, background_count(mix.w, T_bg))
    ks = first_match(mix.w, q, lam2)
    matched = ks >= 0
    a1 = f(1) - alpha
    w = mix.w.copy()
    mu = mix.mu.copy()
    v = mix.v.copy()
    clamp = np.zeros(q.shape[1:], np.bool_)
    for k in range(K):
        hit = matched & (ks == k)
        w[k] = np.where(hit, a1 * mix.w[k] + alpha, a1 * mix.w[k])
        mu_new = np.empty_like(mix.mu[k])
        for c in range(C):
            mu_new[c] = mix.mu[k, c] + alpha * (X[c] - mix.mu[k, c])
        e = X[0] - mu_new[0]
        d2n = e * e
        for c in range(1, C):
            e = X[c] - mu_new[c]
            d2n = d2n + e * e
        vt = mix.v[k] + alpha * (d2n - mix.v[k])
        clamp |= hit & (vt < v_min)
        mu[k] = np.where(hit[None], mu_new, mix.mu[k])
        v[k] = np.where(hit, np.maximum(vt, v_min), mix.v[k])
    rep = ~matched
    w[K - 1] = np.where(rep, w_init, w[K - 1])
    mu[K - 1] = np.where(rep[None], X, mu[K - 1])
    v[K - 1] = np.where(rep, v_init, v[K - 1])
    S = w[0].copy()
    for k in range(1, K):
        S = S + w[k]
    w = w / S[None]
    order = np.argsort(-(w / np.sqrt(v)), axis=0, kind="stable")
    new = type(mix)(np.take_along_axis(w, order, 0), np.take_along_axis(mu, order[:, None], 0),
                    np.take_along_axis(v, order, 0))
    out = type(mix)(np.where(active[None], new.w, mix.w), np.where(active[None, None], new.mu, mix.mu),
                    np.where(active[None], new.v, mix.v))
    return out, used, delta, a, np.where(active, ks, -1), clamp & active, order


def record_window(rgb, depth, p: GmmParams, theta=None):
    """fp32 forward of the Sec. 3.1 GMM over frames [T,H,W,3]/[T,H,W] from a fresh model
    (R-11, R-21), the same operations as oracle.gmm, recording the decisions.

    Returns (Z [T,H,W] float32, has_term [T,H,W] bool, colour Decisions, depth Decisions)."""
    T, H, W = depth.shape
    f = np.float32
    alpha, lam, wd = (f(v) for v in (theta if theta is not None else (p.alpha, p.lam, p.w_depth)))
    lam2 = lam * lam
    mc = fresh_mixture(p.Kc, 3, H, W, f(p.v_init_c), np.float32)
    md = fresh_mixture(p.Kd, 1, H, W, f(p.v_init_d), np.float32)
    Z = np.zeros((T, H, W), f)
    has = np.zeros((T, H, W), np.bool_)

    def empty(K):
        return Decisions(np.zeros((T, H, W), bool), np.zeros((T, H, W), np.int64), np.zeros((T, H, W), bool),
                         np.zeros((T, H, W), np.int64), np.zeros((T, H, W), bool), np.zeros((T, K, H, W), np.int64))
    dc, dd = empty(p.Kc), empty(p.Kd)
    ones = np.ones((H, W), bool)
    for t in range(T):
        Xc = np.moveaxis(rgb[t], -1, 0).astype(f)
        Xd = depth_q8(depth[t], p.depth_max_mm).astype(f)[None]
        valid = depth[t] > 0
        mc, used_c, del_c, a_c, k_c, cl_c, pc = _record_model_step(
            mc, Xc, ones, alpha, lam2, f(p.T_bg), f(p.w_init), f(p.v_init_c), f(p.v_min_c))
        md, used_d, del_d, a_d, k_d, cl_d, pd = _record_model_step(
            md, Xd, valid, alpha, lam2, f(p.T_bg), f(p.w_init), f(p.v_init_d), f(p.v_min_d))
        tc_on, td_on = used_c, valid & used_d
        tc = del_c - lam2
        td = wd * (del_d - lam2)
        Z[t] = np.where(tc_on, np.where(td_on, tc + td, tc), np.where(td_on, td, f(0)))
        has[t] = tc_on | td_on
        for dec, on, a, act, ks, cl, perm in ((dc, tc_on, a_c, ones, k_c, cl_c, pc),
                                               (dd, td_on, a_d, valid, k_d, cl_d, pd)):
            dec.term[t], dec.argmin[t], dec.active[t] = on, a, act
            dec.kstar[t], dec.clamp[t], dec.perm[t] = ks, cl, perm
    return Z, has, dc, dd


def _replay_model(mu, v, X, dec: Decisions, t, alpha, v_init, v_min, tape=None):
    """Continuous part of one model's step with frozen decisions (any precision)."""
    K, C = mu.shape[0], mu.shape[1]
    ks, act = dec.kstar[t], dec.active[t]
    mu_n, v_n = mu.copy(), v.copy()
    for k in range(K):
        hit = act & (ks == k)
        mnew = mu[k] + alpha * (X - mu[k])
        d2n = ((X - mnew) ** 2).sum(0)
        vt = v[k] + alpha * (d2n - v[k])
        mu_n[k] = np.where(hit[None], mnew, mu[k])
        v_n[k] = np.where(hit, np.where(dec.clamp[t], v_min, vt), v[k])
    rep = act & (ks < 0)
    mu_n[K - 1] = np.where(rep[None], X, mu_n[K - 1])
    v_n[K - 1] = np.where(rep, v_init, v_n[K - 1])
    perm = dec.perm[t]
    mu_s = np.take_along_axis(mu_n, perm[:, None], 0)
    v_s = np.take_along_axis(v_n, perm, 0)
    mu_o = np.where(act[None, None], mu_s, mu)
    v_o = np.where(act[None], v_s, v)
    return mu_o, v_o


def _delta(mu, v, X, a):
    m = np.take_along_axis(mu, a[None, None], 0)[0]
    vv = np.take_along_axis(v, a[None], 0)[0]
    return ((X - m) ** 2).sum(0) / vv, m, vv


def replay_window(rgb, depth, p: GmmParams, dc: Decisions, dd: Decisions, theta, dtype=np.float64,
                  keep_tape=False):
    """Z_t(theta), the pre-update score of R-09, with the recorded decisions held fixed (the
    continuous part of the Sec. 3.1 step).  Returns Z [T,H,W] (and the tape of
    pre-step means/variances if keep_tape)."""
    T, H, W = depth.shape
    alpha, lam, wd = (dtype(v) for v in theta)
    lam2 = lam * lam
    muc = np.zeros((p.Kc, 3, H, W), dtype)
    vc = np.full((p.Kc, H, W), p.v_init_c, dtype)
    mud = np.zeros((p.Kd, 1, H, W), dtype)
    vd = np.full((p.Kd, H, W), p.v_init_d, dtype)
    Z = np.zeros((T, H, W), dtype)
    tape = []
    for t in range(T):
        Xc = np.moveaxis(rgb[t], -1, 0).astype(dtype)
        Xd = depth_q8(depth[t], p.depth_max_mm).astype(dtype)[None]
        if keep_tape:
            tape.append((muc, vc, mud, vd, Xc, Xd))
        del_c = _delta(muc, vc, Xc, dc.argmin[t])[0]
        del_d = _delta(mud, vd, Xd, dd.argmin[t])[0]
        tc = del_c - lam2
        td = wd * (del_d - lam2)
        Z[t] = np.where(dc.term[t], np.where(dd.term[t], tc + td, tc), np.where(dd.term[t], td, 0))
        muc, vc = _replay_model(muc, vc, Xc, dc, t, alpha, dtype(p.v_init_c), dtype(p.v_min_c))
        mud, vd = _replay_model(mud, vd, Xd, dd, t, alpha, dtype(p.v_init_d), dtype(p.v_min_d))
    return (Z, tape) if keep_tape else Z


def bce_loss_and_grad(Z, has, gt, t0=1, tau=1.0):
    """The window loss of R-21: mean BCE of sigmoid(Z/tau) against gt (0/255) over frames
    t >= t0 where Z is defined.
    Returns (loss, dL/dZ)."""
    sel = np.zeros_like(has)
    sel[t0:] = has[t0:]
    n = max(int(sel.sum()), 1)
    y = (np.asarray(gt) != 0).astype(Z.dtype)
    s = Z / tau
    # log(1 + exp(s)) - y s, stably
    l = np.maximum(s, 0) - s * y + np.log1p(np.exp(-np.abs(s)))
    loss = float((l * sel).sum() / n)
    sig = 0.5 * (1.0 + np.tanh(0.5 * s))
    g = np.where(sel, (sig - y) / (tau * n), 0.0).astype(Z.dtype)
    return loss, g


def reverse_gradient(rgb, depth, p: GmmParams, dc: Decisions, dd: Decisions, theta, dZ):
    """Hand-written reverse sweep in fp64 of replay_window (chain rule through the mean and
    variance recursions of Sec. 3.1, choices fixed): dL/dtheta = (d alpha, d lambda, d w_d)
    given dL/dZ."""
    f = np.float64
    alpha, lam, wd = (f(v) for v in theta)
    lam2 = lam * lam
    T = depth.shape[0]
    _, tape = replay_window(rgb, depth, p, dc, dd, theta, f, keep_tape=True)
    g_alpha = g_lam = g_wd = 0.0
    a_muc = a_vc = a_mud = a_vd = None
    for t in range(T - 1, -1, -1):
        muc, vc, mud, vd, Xc, Xd = tape[t]
        if a_muc is None:
            a_muc, a_vc = np.zeros_like(muc), np.zeros_like(vc)
            a_mud, a_vd = np.zeros_like(mud), np.zeros_like(vd)
        # state update: adjoint of post-state (a_*) -> pre-state
        a_muc, a_vc, ga = _reverse_model(muc, vc, Xc, dc, t, alpha, a_muc, a_vc)
        g_alpha += ga
        a_mud, a_vd, ga = _reverse_model(mud, vd, Xd, dd, t, alpha, a_mud, a_vd)
        g_alpha += ga
        # score Z_t on the pre-state
        gz = dZ[t].astype(f)
        del_c, mc, vvc = _delta(muc, vc, Xc, dc.argmin[t])
        del_d, md, vvd = _delta(mud, vd, Xd, dd.argmin[t])
        on_c, on_d = dc.term[t], dd.term[t]
        g_lam += float((gz * (-2.0 * lam) * (on_c + wd * on_d)).sum())
        g_wd += float((gz * np.where(on_d, del_d - lam2, 0.0)).sum())
        for on, coef, mu, v, X, a, dl, a_mu, a_v in ((on_c, 1.0, muc, vc, Xc, dc.argmin[t], del_c, a_muc, a_vc),
                                                        (on_d, wd, mud, vd, Xd, dd.argmin[t], del_d, a_mud, a_vd)):
            gd = np.where(on, gz * coef, 0.0)
            m = np.take_along_axis(mu, a[None, None], 0)[0]
            vv = np.take_along_axis(v, a[None], 0)[0]
            for k in range(mu.shape[0]):
                sel = (a == k)
                a_mu[k] += np.where(sel[None], gd[None] * (-2.0) * (X - m) / vv[None], 0.0)
                a_v[k] += np.where(sel, gd * (-dl / vv), 0.0)
    return np.array([g_alpha, g_lam, g_wd])


def _reverse_model(mu, v, X, dec: Decisions, t, alpha, a_mu_out, a_v_out):
    """Adjoint of one model's continuous step (pre-state mu, v; decisions at t)."""
    K = mu.shape[0]
    act = dec.active[t]
    perm = dec.perm[t]
    # un-rank: post-state rank r holds pre-rank perm[r]
    a_mun = np.zeros_like(a_mu_out)
    a_vn = np.zeros_like(a_v_out)
    for r in range(K):
        for k in range(K):
            sel = act & (perm[r] == k)
            a_mun[k] += np.where(sel[None], a_mu_out[r], 0.0)
            a_vn[k] += np.where(sel, a_v_out[r], 0.0)
    ks = dec.kstar[t]
    a_mu = np.where(act[None, None], 0.0, a_mu_out)
    a_v = np.where(act[None], 0.0, a_v_out)
    g_alpha = 0.0
    for k in range(K):
        hit = act & (ks == k)
        rep = act & (ks < 0) & (k == K - 1)
        keep = act & ~hit & ~rep
        a_mu[k] += np.where(keep[None], a_mun[k], 0.0)
        a_v[k] += np.where(keep, a_vn[k], 0.0)
        # matched: mu' = mu + alpha (X - mu); v~ = v + alpha(|X - mu'|^2 - v)
        mnew = mu[k] + alpha * (X - mu[k])
        d2n = ((X - mnew) ** 2).sum(0)
        av = np.where(hit & ~dec.clamp[t], a_vn[k], 0.0)
        a_mnew = a_mun[k] + av[None] * alpha * (-2.0) * (X - mnew)
        a_mu[k] += np.where(hit[None], (1.0 - alpha) * a_mnew, 0.0)
        a_v[k] += np.where(hit, (1.0 - alpha) * av, 0.0)
        g_alpha += float(np.where(hit, av * (d2n - v[k]), 0.0).sum())
        g_alpha += float(np.where(hit[None], a_mnew * (X - mu[k]), 0.0).sum())
    return a_mu, a_v, g_alpha


def window_loss(rgb, depth, gt, p: GmmParams, dc, dd, has, theta, t0=1, tau=1.0):
    """The R-21 loss of the fp64 replay at theta (decisions frozen)."""
    Z = replay_window(rgb, depth, p, dc, dd, theta, np.float64)
    return bce_loss_and_grad(Z, has, gt, t0, tau)[0]


def fd_gradient(rgb, depth, gt, p: GmmParams, dc, dd, has, theta, rel_h=1e-6):
    """Central differences of the replayed fp64 loss (decisions frozen)."""
    g = np.zeros(3)
    th = np.array(theta, np.float64)
    for i in range(3):
        h = rel_h * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        g[i] = (window_loss(rgb, depth, gt, p, dc, dd, has, tp) -
                window_loss(rgb, depth, gt, p, dc, dd, has, tm)) / (2 * h)
    return g
