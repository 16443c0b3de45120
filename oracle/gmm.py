"""RGB-D Gaussian mixture background model: one classify-and-update step per frame.

Oracle (test infrastructure only).  Plain numpy, vectorised over pixels,
explicit loops over mixture components, every operation rounded on its own in
the order written below.  ``dtype`` selects IEEE binary32 (parity with the
GPU) or binary64 (gradient reference).

What the paper fixes (Sec. 3.1) and what is read in
------------------------------------------------------
* Each pixel carries its own mixture of k Gaussians (omega, mu, sigma^2): a
  normalised weight, a mean per colour component and one variance per
  Gaussian (Sec. 3.1, first paragraph; the "three variances" remark is read as
  the independence assumption, so one isotropic variance per component).
* The RGB-D variant keeps two separate mixtures, a 3-channel colour model and
  a 1-channel depth model, and combines their results (Sec. 3.1, second
  paragraph).  The depth model is used only where the sensor depth is > 0;
  elsewhere the pixel is classified by colour alone (Sec. 3.1, end).
* The base algorithm is the Stauffer-Grimson online mixture (cited, not
  restated, in Sec. 3.1): a sample matches a Gaussian within lambda standard
  deviations; matched weight += alpha(1 - w), others decay; the matched mean
  and variance follow with rate rho; with no match the weakest Gaussian is
  replaced; Gaussians are ranked by omega/sigma and the leading ones whose
  weights add up past T_bg form the background.
* Classification uses the density of Eq. (1) for both models and the product
  of the two factors (Sec. 3.1); the decision diagram (Fig. 1) is not
  available.  Reading: taking the log of the product and keeping the exponent
  terms, each model contributes its smallest normalised squared distance
  delta_m = min over background Gaussians of d^2/sigma^2, and the pixel is
  foreground when Z = (delta_c - lambda^2) + w_d * (delta_d - lambda^2) >= 0.
  With no valid depth (or w_d = 0) this is exactly the Stauffer-Grimson test
  "the pixel matches none of the background Gaussians".

Variance variant (``var_mode`` 1; R-05 keeps one isotropic variance): the other
reading of Sec. 3.1's remark that independent colour components allow three
variances instead of a covariance matrix.  Each colour Gaussian has a variance per
channel; q_k = ((e_0^2/v_0 + e_1^2/v_1) + e_2^2/v_2), each term rounded as
written (the squared Mahalanobis distance), matched when q_k < lambda^2; each
channel's variance follows its own squared deviation from the new mean and is
floored on its own; new Gaussians start, and variances are floored, at one third of
the isotropic constants (the isotropic v is the sum of the three); the rank key is
w / sqrt((v_0 + v_1) + v_2), and where a single variance is needed (the Eq. (1)
density) it is that sum.  The depth model has one channel and is unchanged.

Decision variant (``decision`` 1; R-09 keeps the exponent terms only): each model's
factor is Eq. (1) scaled by s for the background Gaussian that attains delta_m,
P_m = s * exp(-delta_m / 2) / (2 pi v), v that Gaussian's variance (binary32 in
the order exp, 2 pi * v, division, scaling); the product P = P_c * P_d where the
depth term is present (else the single factor), and the pixel is foreground when
P < tau.  Parity unpinned beyond its agreement with the log-sum rule when tau is
set from equal variances (tests).

Update rate of the matched mean and variance (R-06 and its variants): rho = alpha
(``rho_mode`` 0), or rho = alpha / w_k* with w_k* the matched weight after its
update and before renormalisation (``rho_mode`` 1; the rule of OpenCV's mixture
model, which Sec. 3.1 names as a basis of the authors' GMM), or rho = alpha * eta
with eta the Eq. (1) density of the matched Gaussian at the sample,
exp(-q/2) / (2 pi v) before its update (``rho_mode`` 2; Stauffer-Grimson's own
rate).

Per-pixel step (both models; X is the model's input vector, C its channel
count, a = 1 - alpha, rho as above, lam2 = lambda*lambda):

  distances  e = X - mu_k;  d2_k = ((e0*e0) + e1*e1) + e2*e2  (C = 3) or e0*e0;
             q_k = d2_k / v_k
  decision   (on the pre-update model) used = w_0 > 0;  B = smallest b with
             w_0 + ... + w_{b-1} > T_bg (summed in order), else the number of
             Gaussians with w > 0;  delta = min_{k < B} q_k
  match      k* = first k (rank order) with w_k > 0 and q_k < lam2
  matched    w_k = a*w_k (k != k*);  w_k* = (a*w_k*) + alpha;
             mu_k* = mu_k* + rho*(X - mu_k*);
             v_k* = v_k* + rho*(||X - mu_k*(new)||^2 - v_k*);  v_k* = max(v_k*, v_min)
  unmatched  w_k = a*w_k for all k, then Gaussian K-1 = (w_init, X, v_init)
  normalise  S = ((w_0 + w_1) + ...);  w_k = w_k / S
  rank       stable sort by w_k / sqrt(v_k), descending

Mask: 255 where Z >= 0, 0 elsewhere and where no model has data yet.  The
colour model is updated every frame; the depth model only where depth > 0.
Fresh state: w = 0, mu = 0, v = v_init, so frame 0 seeds every pixel through
the "unmatched" branch.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .depth import DEPTH_MAX_MM, depth_q8, depth_valid


@dataclass
class GmmParams:
    """Model constants.  Defaults are the readings listed in the module docstring.

    Sec. 3.1 quotes 7 colour / 3 depth Gaussians and a learning rate of 0.001 for
    the authors' own system; the workloads here use K = 3 or 5 and alpha = 0.01.
    """
    Kc: int = 3
    Kd: int = 3
    alpha: float = 0.01
    lam: float = 2.5
    T_bg: float = 0.7
    w_init: float = 0.05
    v_init_c: float = 675.0   # (15 grey levels)^2 in each of 3 channels
    v_min_c: float = 12.0     # (2 levels)^2 in each of 3 channels
    v_init_d: float = 25.0    # 5 depth codes (about 20 cm)
    v_min_d: float = 1.0      # 1 depth code (about 4 cm, Sec. 4.2)
    w_depth: float = 1.0
    depth_max_mm: int = DEPTH_MAX_MM
    rho_mode: int = 0          # 0: alpha; 1: alpha / w (matched, updated); 2: alpha * eta
    decision: int = 0          # 0: Z = (d_c - lam^2) + w_d (d_d - lam^2) >= 0; 1: P < tau
    density_scale: float = 10000.0   # s (Sec. 3.1 default)
    density_threshold: float = 1.0   # tau
    var_mode: int = 0          # 0: one variance per colour Gaussian; 1: one per channel


@dataclass
class Mixture:
    """One model's per-pixel mixture (Sec. 3.1: K Gaussians per pixel, each a weight, a
    mean and a variance): w [K,H,W], mu [K,C,H,W], v [K,H,W]."""
    w: np.ndarray
    mu: np.ndarray
    v: np.ndarray

    def copy(self) -> "Mixture":
        """An independent copy of the three arrays."""
        return Mixture(self.w.copy(), self.mu.copy(), self.v.copy())


def fresh_mixture(K: int, C: int, H: int, W: int, v_init, dtype) -> Mixture:
    """The model before the first frame (R-11; Sec. 3.1 gives no initialisation): every
    weight 0, every mean 0, every variance v_init."""
    return Mixture(np.zeros((K, H, W), dtype), np.zeros((K, C, H, W), dtype),
                   np.full((K, H, W), v_init, dtype))


def fresh_mixture_diag(K: int, C: int, H: int, W: int, v_init, dtype) -> Mixture:
    """A mixture with a variance per channel (R-05', the other reading of Sec. 3.1's
    three-variances remark): v [K,C,H,W]."""
    return Mixture(np.zeros((K, H, W), dtype), np.zeros((K, C, H, W), dtype),
                   np.full((K, C, H, W), v_init, dtype))


def mahalanobis_sq(mix: Mixture, X: np.ndarray) -> np.ndarray:
    """q[k] = sum over channels, in channel order, of (X - mu_k)^2 / v_k (per-channel v)."""
    K, C = mix.mu.shape[0], mix.mu.shape[1]
    q = np.empty((K,) + X.shape[1:], X.dtype)
    for k in range(K):
        e = X[0] - mix.mu[k, 0]
        acc = (e * e) / mix.v[k, 0]
        for c in range(1, C):
            e = X[c] - mix.mu[k, c]
            acc = acc + (e * e) / mix.v[k, c]
        q[k] = acc
    return q


def variance_sum(v: np.ndarray) -> np.ndarray:
    """The single variance of a Gaussian: v itself, or ((v_0 + v_1) + ...) if per channel."""
    if v.ndim == 3:
        return v
    acc = v[:, 0]
    for c in range(1, v.shape[1]):
        acc = acc + v[:, c]
    return acc


def sq_distances(mix: Mixture, X: np.ndarray) -> np.ndarray:
    """d2[k] = sum over channels, in channel order, of (X - mu_k)^2.  X: [C,H,W]."""
    K, C = mix.mu.shape[0], mix.mu.shape[1]
    d2 = np.empty((K,) + X.shape[1:], X.dtype)
    for k in range(K):
        e = X[0] - mix.mu[k, 0]
        acc = e * e
        for c in range(1, C):
            e = X[c] - mix.mu[k, c]
            acc = acc + e * e
        d2[k] = acc
    return d2


def background_count(w: np.ndarray, T_bg) -> np.ndarray:
    """B: the smallest b whose leading weights sum (in order) past T_bg, else #(w > 0)."""
    K = w.shape[0]
    B = (w > 0).sum(axis=0).astype(np.int64)
    found = np.zeros(w.shape[1:], np.bool_)
    cum = np.zeros(w.shape[1:], w.dtype)
    for k in range(K):
        cum = cum + w[k]
        hit = ~found & (cum > T_bg)
        B[hit] = k + 1
        found |= hit
    return B


def background_distance(q: np.ndarray, B: np.ndarray) -> np.ndarray:
    """delta = min over the B background Gaussians of q_k (defined where B >= 1)."""
    return background_argmin(q, B)[0]


def background_argmin(q: np.ndarray, B: np.ndarray):
    """(delta, k): the minimum over the B background Gaussians and the first index attaining it."""
    delta = q[0].copy()
    arg = np.zeros(q.shape[1:], np.int64)
    for k in range(1, q.shape[0]):
        better = (k < B) & (q[k] < delta)
        delta = np.where(better, q[k], delta)
        arg = np.where(better, k, arg)
    return delta, arg


def density_factor(delta: np.ndarray, v: np.ndarray, s) -> np.ndarray:
    """s * exp(-delta/2) / (2 pi v): Eq. (1) scaled by s, for the Gaussian attaining delta."""
    f = delta.dtype.type
    e = np.exp(f(-0.5) * delta)
    return f(s) * (e / (f(2.0 * np.pi) * v))


def first_match(w: np.ndarray, q: np.ndarray, lam2) -> np.ndarray:
    """k*: first Gaussian in rank order with w > 0 and q < lambda^2; -1 if none."""
    ks = np.full(w.shape[1:], -1, np.int64)
    for k in range(w.shape[0] - 1, -1, -1):
        ks = np.where((w[k] > 0) & (q[k] < lam2), k, ks)
    return ks


def update_mixture(mix: Mixture, X: np.ndarray, q: np.ndarray, active: np.ndarray,
                   alpha, lam2, w_init, v_init, v_min, rho_mode: int = 0) -> Mixture:
    """Stauffer-Grimson update + replacement + renormalisation + ranking where ``active``."""
    f = mix.w.dtype.type
    K, C = mix.mu.shape[0], mix.mu.shape[1]
    diag = mix.v.ndim == 4          # a variance per channel
    vsum = variance_sum(mix.v)
    a = f(1) - alpha
    ks = first_match(mix.w, q, lam2)
    matched = ks >= 0
    w = mix.w.copy()
    mu = mix.mu.copy()
    v = mix.v.copy()
    for k in range(K):
        hit = matched & (ks == k)
        w[k] = np.where(hit, a * mix.w[k] + alpha, a * mix.w[k])
        # rho is used only where hit (there w >= alpha > 0)
        if rho_mode == 1:
            rho = alpha / np.where(hit, w[k], f(1))
        elif rho_mode == 2:
            with np.errstate(under="ignore"):
                rho = alpha * (np.exp(f(-0.5) * q[k]) / (f(2.0 * np.pi) * vsum[k]))
        else:
            rho = alpha
        mu_new = np.empty_like(mix.mu[k])
        for c in range(C):
            mu_new[c] = mix.mu[k, c] + rho * (X[c] - mix.mu[k, c])
        if diag:
            v_new = np.empty_like(mix.v[k])
            for c in range(C):
                e = X[c] - mu_new[c]
                v_new[c] = np.maximum(mix.v[k, c] + rho * (e * e - mix.v[k, c]), v_min)
            v[k] = np.where(hit[None], v_new, mix.v[k])
        else:
            e = X[0] - mu_new[0]
            d2n = e * e
            for c in range(1, C):
                e = X[c] - mu_new[c]
                d2n = d2n + e * e
            v_new = mix.v[k] + rho * (d2n - mix.v[k])
            v_new = np.maximum(v_new, v_min)
            v[k] = np.where(hit, v_new, mix.v[k])
        mu[k] = np.where(hit[None], mu_new, mix.mu[k])
    # No match: the last-ranked Gaussian is replaced by a new one centred on X.
    rep = ~matched
    w[K - 1] = np.where(rep, w_init, w[K - 1])
    mu[K - 1] = np.where(rep[None], X, mu[K - 1])
    v[K - 1] = np.where(rep[None] if diag else rep, v_init, v[K - 1])
    # Renormalise (sequential sum) and rank by omega/sigma (stable, descending).
    S = w[0].copy()
    for k in range(1, K):
        S = S + w[k]
    w = w / S[None]
    key = w / np.sqrt(variance_sum(v))
    order = np.argsort(-key, axis=0, kind="stable")
    w = np.take_along_axis(w, order, axis=0)
    v = np.take_along_axis(v, order[:, None] if diag else order, axis=0)
    mu = np.take_along_axis(mu, order[:, None], axis=0)
    out = Mixture(np.where(active[None], w, mix.w), np.where(active[None, None], mu, mix.mu),
                  np.where(active[None, None] if diag else active[None], v, mix.v))
    return out


class GmmRef:
    """The RGB-D GMM over an H x W image (Sec. 3.1: a colour and a depth mixture per
    pixel, combined in the decision).  ``step(rgb, depth) -> mask``."""

    def __init__(self, H: int, W: int, params: GmmParams | None = None, dtype=np.float32):
        self.p = params or GmmParams()
        self.H, self.W = H, W
        self.dtype = np.dtype(dtype)
        f = self.dtype.type
        if self.p.var_mode == 1:
            self.colour = fresh_mixture_diag(self.p.Kc, 3, H, W, f(self.p.v_init_c) / f(3), self.dtype)
        else:
            self.colour = fresh_mixture(self.p.Kc, 3, H, W, f(self.p.v_init_c), self.dtype)
        self.depth = fresh_mixture(self.p.Kd, 1, H, W, f(self.p.v_init_d), self.dtype)
        self.t = 0
        self.last_Z = None
        self.last_P = None
        self.last_has_term = None

    def constants(self):
        """The parameters in the working precision (each rounded once, as the kernels do)."""
        f = self.dtype.type
        p = self.p
        return dict(alpha=f(p.alpha), lam=f(p.lam), T_bg=f(p.T_bg), w_init=f(p.w_init),
                    v_init_c=f(p.v_init_c), v_min_c=f(p.v_min_c), v_init_d=f(p.v_init_d),
                    v_min_d=f(p.v_min_d), w_depth=f(p.w_depth))

    def step(self, rgb: np.ndarray, depth: np.ndarray) -> np.ndarray:
        """One frame (Sec. 3.1): both mixtures' distances, the decision on the pre-update
        models (R-08, R-09, or R-09' with `decision` 1), then each active model's match,
        update, replacement, renormalisation and ranking (R-06..R-08, R-10, R-12)."""
        c = self.constants()
        f = self.dtype.type
        lam2 = c["lam"] * c["lam"]
        Xc = np.moveaxis(np.asarray(rgb), -1, 0).astype(self.dtype)            # [3,H,W]
        Xd = depth_q8(depth, self.p.depth_max_mm).astype(self.dtype)[None]     # [1,H,W]
        valid = depth_valid(depth)

        diag = self.p.var_mode == 1
        qc = mahalanobis_sq(self.colour, Xc) if diag else sq_distances(self.colour, Xc) / self.colour.v
        qd = sq_distances(self.depth, Xd) / self.depth.v

        # Decision on the pre-update (ranked) models.
        used_c = self.colour.w[0] > 0
        used_d = self.depth.w[0] > 0
        dc, kc = background_argmin(qc, background_count(self.colour.w, c["T_bg"]))
        dd, kd = background_argmin(qd, background_count(self.depth.w, c["T_bg"]))
        term_c = used_c
        term_d = valid & used_d
        tc = dc - lam2
        td = c["w_depth"] * (dd - lam2)
        Z = np.where(term_c, np.where(term_d, tc + td, tc), td)
        has_term = term_c | term_d
        if self.p.decision == 1:
            vc = np.take_along_axis(variance_sum(self.colour.v), kc[None], axis=0)[0]
            vd = np.take_along_axis(self.depth.v, kd[None], axis=0)[0]
            with np.errstate(over="ignore", under="ignore"):
                Pc = density_factor(dc, vc, self.p.density_scale)
                Pd = density_factor(dd, vd, self.p.density_scale)
                P = np.where(term_c, np.where(term_d, Pc * Pd, Pc), Pd)
            mask = np.where(has_term & (P < f(self.p.density_threshold)), 255, 0).astype(np.uint8)
            self.last_P = np.where(has_term, P, f(0))
        else:
            mask = np.where(has_term & (Z >= 0), 255, 0).astype(np.uint8)
        self.last_Z = np.where(has_term, Z, f(0))
        self.last_has_term = has_term

        ones = np.ones((self.H, self.W), np.bool_)
        rm = self.p.rho_mode
        vi_c, vm_c = (c["v_init_c"] / f(3), c["v_min_c"] / f(3)) if diag else (c["v_init_c"], c["v_min_c"])
        self.colour = update_mixture(self.colour, Xc, qc, ones, c["alpha"], lam2, c["w_init"],
                                     vi_c, vm_c, rm)
        self.depth = update_mixture(self.depth, Xd, qd, valid, c["alpha"], lam2, c["w_init"],
                                    c["v_init_d"], c["v_min_d"], rm)
        self.t += 1
        return mask

    # State in the library's canonical plane order (see include/fgs.h).
    def state_planes(self) -> dict:
        """The state in the library's serialised plane order (fgs_copy_state's payload)."""
        return dict(w_c=self.colour.w, mu_c=self.colour.mu, v_c=self.colour.v,
                    w_d=self.depth.w, mu_d=self.depth.mu[:, 0], v_d=self.depth.v, t=self.t)

    def set_state_planes(self, st: dict) -> None:
        """Replace the state from planes in that order (fgs_set_state's payload)."""
        dt = self.dtype
        self.colour = Mixture(np.array(st["w_c"], dt), np.array(st["mu_c"], dt), np.array(st["v_c"], dt))
        self.depth = Mixture(np.array(st["w_d"], dt), np.array(st["mu_d"], dt)[:, None],
                             np.array(st["v_d"], dt))
        self.t = int(st.get("t", 0))
