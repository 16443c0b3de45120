"""The oracle's pins catch plausible mistakes.  Each case plants one mistake in the oracle
(a dropped term, a wrong sign, index, operand or order; the function's source rewritten
in one place), then runs that model's pin tests: at least one must fail.  The mistakes
live only in the test's patched copy; nothing here runs on the GPU."""
import inspect
import textwrap

import numpy as np
import pytest

import oracle.adjoint
import oracle.depth
import oracle.gmm
import oracle.metrics
import oracle.pbas
import oracle.philox
import oracle.postfilter
import oracle.static
import test_oracle_adjoint
import test_oracle_depth
import test_oracle_gmm
import test_oracle_metrics
import test_oracle_pbas
import test_oracle_pbas_gradient
import test_oracle_philox
import test_oracle_postfilter
import test_oracle_static


def _mutant(func, old, new):
    """`func` with its source changed in one place, compiled in its module's namespace."""
    src = textwrap.dedent(inspect.getsource(func))
    assert src.count(old) == 1, (func.__qualname__, old)
    ns = dict(inspect.getmodule(func).__dict__)
    exec(compile(src.replace(old, new), f"<mutant of {func.__qualname__}>", "exec"), ns)
    return ns[func.__name__]


def _patch(monkeypatch, owner, name, new, test_modules):
    """Replace owner.name, and every test module's own reference to the same object."""
    orig = getattr(owner, name)
    monkeypatch.setattr(owner, name, new)
    for tm in test_modules:
        for attr, val in list(vars(tm).items()):
            if val is orig:
                monkeypatch.setattr(tm, attr, new)


def _pin_calls(mod):
    """Every test function of a pin module with each of its parametrizations."""
    calls = []
    for name, fn in vars(mod).items():
        if not name.startswith("test_") or not callable(fn):
            continue
        params = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        if not params:
            if not inspect.signature(fn).parameters:
                calls.append((name, fn, {}))
            continue
        argnames = [a.strip() for a in params[0].args[0].split(",")]
        for vals in params[0].args[1]:
            vals = vals if len(argnames) > 1 else (vals,)
            calls.append((name, fn, dict(zip(argnames, vals))))
    return calls


def _caught(mod):
    """Name of the first pin that fails (None if all pass)."""
    for name, fn, kw in _pin_calls(mod):
        try:
            with np.errstate(all="ignore"):
                fn(**kw)
        except Exception:   # an assertion, or the planted mistake breaking the run
            return name
    return None


GMM_MUTANTS = [
    ("variance from the old mean", oracle.gmm, "update_mixture",
     "            e = X[0] - mu_new[0]", "            e = X[0] - mix.mu[k, 0]"),
    ("matched weight misses +alpha", oracle.gmm, "update_mixture",
     "np.where(hit, a * mix.w[k] + alpha, a * mix.w[k])", "np.where(hit, a * mix.w[k], a * mix.w[k])"),
    ("ranking ascending", oracle.gmm, "update_mixture",
     "np.argsort(-key, axis=0", "np.argsort(key, axis=0"),
    ("replacement mean into rank 0", oracle.gmm, "update_mixture",
     "mu[K - 1] = np.where(rep[None], X, mu[K - 1])", "mu[0] = np.where(rep[None], X, mu[0])"),
    ("no renormalisation", oracle.gmm, "update_mixture", "w = w / S[None]", "w = w"),
    ("last channel dropped from d2", oracle.gmm, "sq_distances",
     "for c in range(1, C):", "for c in range(1, max(1, C - 1)):"),
    ("background count off by one", oracle.gmm, "background_count", "B[hit] = k + 1", "B[hit] = k"),
    ("unused Gaussians may match", oracle.gmm, "first_match",
     "(w[k] > 0) & (q[k] < lam2)", "(q[k] < lam2)"),
    ("depth term subtracted", oracle.gmm.GmmRef, "step",
     "Z = np.where(term_c, np.where(term_d, tc + td, tc), td)",
     "Z = np.where(term_c, np.where(term_d, tc - td, tc), td)"),
    ("lambda not squared", oracle.gmm.GmmRef, "step",
     "lam2 = c[\"lam\"] * c[\"lam\"]", "lam2 = c[\"lam\"]"),
    ("no variance floor", oracle.gmm, "update_mixture",
     "v_new = np.maximum(v_new, v_min)", "v_new = v_new"),
    ("last match instead of first", oracle.gmm, "first_match",
     "for k in range(w.shape[0] - 1, -1, -1):", "for k in range(w.shape[0]):"),
    ("depth term without valid depth", oracle.gmm.GmmRef, "step",
     "term_d = valid & used_d", "term_d = used_d"),
    ("rate alpha/w with the weight before its update", oracle.gmm, "update_mixture",
     "rho = alpha / np.where(hit, w[k], f(1))", "rho = alpha / np.where(hit, mix.w[k], f(1))"),
    ("rate alpha*eta without the 2 pi", oracle.gmm, "update_mixture",
     "rho = alpha * (np.exp(f(-0.5) * q[k]) / (f(2.0 * np.pi) * vsum[k]))",
     "rho = alpha * (np.exp(f(-0.5) * q[k]) / vsum[k])"),
    ("density of the first background Gaussian", oracle.gmm.GmmRef, "step",
     "vc = np.take_along_axis(variance_sum(self.colour.v), kc[None], axis=0)[0]",
     "vc = variance_sum(self.colour.v)[0]"),
    ("density decision inverted", oracle.gmm.GmmRef, "step",
     "(P < f(self.p.density_threshold))", "(P > f(self.p.density_threshold))"),
    ("per-channel variances not split", oracle.gmm.GmmRef, "step",
     "(c[\"v_init_c\"] / f(3), c[\"v_min_c\"] / f(3)) if diag", "(c[\"v_init_c\"], c[\"v_min_c\"] / f(3)) if diag"),
]

PBAS_MUTANTS = [
    ("R moves the wrong way", oracle.pbas.PbasRef, "step",
     "self.R > dbar * f(p.R_scale)", "self.R < dbar * f(p.R_scale)"),
    ("T increments swapped", oracle.pbas.PbasRef, "step",
     "np.where(F, self.T + f(p.T_inc) / dbar, self.T - f(p.T_dec) / dbar)",
     "np.where(F, self.T - f(p.T_dec) / dbar, self.T + f(p.T_inc) / dbar)"),
    ("S misses the replaced D", oracle.pbas.PbasRef, "step",
     "self.S[ys, xs, js] += dm - old", "self.S[ys, xs, js] += dm"),
    ("neighbour gets the source's value", oracle.pbas.PbasRef, "step",
     "self.samples[knb[ys, xs, js], ny, nx, js] = I[ny, nx, js]",
     "self.samples[knb[ys, xs, js], ny, nx, js] = I[ys, xs, js]"),
    ("empty depth slots counted", oracle.pbas.PbasRef, "step",
     "filled[..., 3] = s[..., 3] != 0", "filled[..., 3] = True"),
    ("distance equal to R matches", oracle.pbas.PbasRef, "step",
     "cnt += filled & (dist < self.R)", "cnt += filled & (dist <= self.R)"),
    ("one match too many needed", oracle.pbas.PbasRef, "step",
     "F = active & (cnt < p.min_matches)", "F = active & (cnt <= p.min_matches)"),
    ("neighbour offsets transposed", oracle.pbas.PbasRef, "step",
     "ny, nx = ys + NB_DY[d], xs + NB_DX[d]", "ny, nx = ys + NB_DX[d], xs + NB_DY[d]"),
    ("no R floor", oracle.pbas.PbasRef, "step",
     "R_new = np.maximum(R_new, np.array(p.R_lower, f))", "R_new = R_new"),
    ("draws: frame and block swapped in the counter", oracle.pbas, "pbas_draws",
     "philox4x32_10(pix, np.uint64(t), np.uint64(c), np.uint64(0), k0, k1)",
     "philox4x32_10(pix, np.uint64(c), np.uint64(t), np.uint64(0), k0, k1)"),
    ("draws: self and neighbour blocks exchanged", oracle.pbas, "pbas_draws",
     "return out[0], out[1]", "return out[1], out[0]"),
    ("draws: key words exchanged", oracle.pbas, "pbas_draws",
     "k0, k1 = seed_key(seed)", "k1, k0 = seed_key(seed)"),
    ("draws: window keyed by its own width", oracle.pbas, "pbas_draws",
     "pix = ys * np.uint64(W_img) + xs", "pix = ys * np.uint64(W) + xs"),
]

GRADIENT_MUTANTS = [
    ("gradient weight from this frame's mean", oracle.pbas.PbasRef, "_step_gradient",
     "gradient_mean(self.gsum_prev, H * W)", "gradient_mean(gsum, H * W)"),
    ("no floor under the gradient mean", oracle.pbas.PbasRef, "_step_gradient",
     "np.maximum(gradient_mean(self.gsum_prev, H * W), f(1.0))", "gradient_mean(self.gsum_prev, H * W)"),
    ("neighbour keeps its old magnitude", oracle.pbas.PbasRef, "_step_gradient",
     "self.gsamples[kk[c], ny[c], nx[c], js[c]] = M[ny[c], nx[c], js[c]]", "pass"),
    ("self-update keeps the old magnitude", oracle.pbas.PbasRef, "_step_gradient",
     "self.gsamples[ks[c], ys[c], xs[c], js[c]] = M[ys[c], xs[c], js[c]]", "pass"),
    ("Sobel border padded with zeros", oracle.pbas, "sobel_l1_magnitude",
     'np.pad(np.asarray(plane, np.int32), 1, mode="edge")', 'np.pad(np.asarray(plane, np.int32), 1, mode="constant")'),
    ("Sobel y response taken along x", oracle.pbas, "sobel_l1_magnitude",
     "gy = (at(1, -1) + 2 * at(1, 0) + at(1, 1)) - (at(-1, -1) + 2 * at(-1, 0) + at(-1, 1))", "gy = gx"),
    ("gradient S misses the replaced D", oracle.pbas.PbasRef, "_step_gradient",
     "self.S[ys, xs, js] = (self.S[ys, xs, js] - old) + dm", "self.S[ys, xs, js] = self.S[ys, xs, js] + dm"),
    ("gradient term unweighted", oracle.pbas.PbasRef, "_step_gradient",
     "dist[..., :3] = wgt * dm + dv[..., :3]", "dist[..., :3] = dm + dv[..., :3]"),
]

OTHER_MUTANTS = [
    ("static: run must exceed M", oracle.static.StaticRef, "step",
     "self.count >= self.M", "self.count > self.M", test_oracle_static),
    ("static: run not reset by background", oracle.static.StaticRef, "step",
     "np.minimum(self.count + 1, COUNTER_MAX), 0)", "np.minimum(self.count + 1, COUNTER_MAX), self.count)",
     test_oracle_static),
    ("static: counter not saturated", oracle.static.StaticRef, "step",
     "np.minimum(self.count + 1, COUNTER_MAX)", "self.count + 1", test_oracle_static),
    ("depth code rounds down", oracle.depth, "depth_q8", "q = (255 * d + m // 2) // m", "q = (255 * d) // m",
     test_oracle_depth),
    ("upscale takes corners", oracle.depth, "upscale_nearest",
     "ys = ((2 * np.arange(H, dtype=np.int64) + 1) * Hd) // (2 * H)",
     "ys = (np.arange(H, dtype=np.int64) * Hd) // H", test_oracle_depth),
    ("false positives and negatives swapped", oracle.metrics, "indicators",
     "FNR=_div(fn, tp + fn)", "FNR=_div(fp, tp + fn)", test_oracle_metrics),
    ("median border padded with zeros", oracle.postfilter, "median_mask",
     'np.pad(m, r, mode="edge")', 'np.pad(m, r, mode="constant")', test_oracle_postfilter),
    ("median takes the next-larger element", oracle.postfilter, "median_mask",
     "[..., (k * k) // 2]", "[..., (k * k) // 2 + 1]", test_oracle_postfilter),
    ("median treats only values >= 128 as foreground", oracle.postfilter, "median_mask",
     "np.asarray(mask) != 0", "np.asarray(mask) >= 128", test_oracle_postfilter),
    ("median window one row short", oracle.postfilter, "median_mask",
     "padded[a:b + 2 * r]", "padded[a + 1:b + 2 * r]", test_oracle_postfilter),
    ("median window anchored at its left edge", oracle.postfilter, "median_mask",
     'np.pad(m, r, mode="edge")', 'np.pad(m, ((r, r), (0, 2 * r)), mode="edge")', test_oracle_postfilter),
]


ADJOINT_MUTANTS = [
    ("lambda gradient ignores the depth weight", oracle.adjoint, "reverse_gradient",
     "(on_c + wd * on_d)", "(on_c + on_d)"),
    ("alpha gradient misses the variance path", oracle.adjoint, "_reverse_model",
     "g_alpha += float(np.where(hit, av * (d2n - v[k]), 0.0).sum())", "g_alpha += 0.0"),
    ("mean adjoint without the variance's pull", oracle.adjoint, "_reverse_model",
     "a_mnew = a_mun[k] + av[None] * alpha * (-2.0) * (X - mnew)", "a_mnew = a_mun[k]"),
    ("depth weight gradient misses lambda squared", oracle.adjoint, "reverse_gradient",
     "np.where(on_d, del_d - lam2, 0.0)", "np.where(on_d, del_d, 0.0)"),
    ("clamped variance passes its adjoint", oracle.adjoint, "_reverse_model",
     "av = np.where(hit & ~dec.clamp[t], a_vn[k], 0.0)", "av = np.where(hit, a_vn[k], 0.0)"),
]


@pytest.mark.parametrize("what,owner,name,old,new", GMM_MUTANTS, ids=[m[0] for m in GMM_MUTANTS])
def test_gmm_pins_catch(monkeypatch, what, owner, name, old, new):
    _patch(monkeypatch, owner, name, _mutant(getattr(owner, name), old, new), [test_oracle_gmm])
    assert _caught(test_oracle_gmm) is not None, what


@pytest.mark.parametrize("what,owner,name,old,new", PBAS_MUTANTS, ids=[m[0] for m in PBAS_MUTANTS])
def test_pbas_pins_catch(monkeypatch, what, owner, name, old, new):
    _patch(monkeypatch, owner, name, _mutant(getattr(owner, name), old, new), [test_oracle_pbas])
    assert _caught(test_oracle_pbas) is not None, what


@pytest.mark.parametrize("what,owner,name,old,new", GRADIENT_MUTANTS, ids=[m[0] for m in GRADIENT_MUTANTS])
def test_gradient_pins_catch(monkeypatch, what, owner, name, old, new):
    _patch(monkeypatch, owner, name, _mutant(getattr(owner, name), old, new), [test_oracle_pbas_gradient])
    assert _caught(test_oracle_pbas_gradient) is not None, what


@pytest.mark.parametrize("what,owner,name,old,new,pins", OTHER_MUTANTS, ids=[m[0] for m in OTHER_MUTANTS])
def test_other_pins_catch(monkeypatch, what, owner, name, old, new, pins):
    _patch(monkeypatch, owner, name, _mutant(getattr(owner, name), old, new), [pins])
    assert _caught(pins) is not None, what


@pytest.mark.parametrize("what,owner,name,old,new", ADJOINT_MUTANTS, ids=[m[0] for m in ADJOINT_MUTANTS])
def test_adjoint_pins_catch(monkeypatch, what, owner, name, old, new):
    _patch(monkeypatch, owner, name, _mutant(getattr(owner, name), old, new), [test_oracle_adjoint])
    assert _caught(test_oracle_adjoint) is not None, what


def test_philox_pin_catches_swapped_key_words(monkeypatch, rocrand_probe):
    # a round that xors the key words into the wrong lanes: only the library comparison can
    # see it (the two oracle implementations share nothing but the constants)
    bad = _mutant(oracle.philox.philox4x32_10,
                  "c = [hi1 ^ c[1] ^ np.uint64(ka), lo1, hi0 ^ c[3] ^ np.uint64(kb), lo0]",
                  "c = [hi1 ^ c[1] ^ np.uint64(kb), lo1, hi0 ^ c[3] ^ np.uint64(ka), lo0]")
    _patch(monkeypatch, oracle.philox, "philox4x32_10", bad, [test_oracle_philox])
    with pytest.raises(AssertionError):
        test_oracle_philox.test_matches_rocm_library(rocrand_probe)


def test_unmutated_oracle_passes_its_pins():
    for mod in (test_oracle_gmm, test_oracle_pbas, test_oracle_depth, test_oracle_metrics, test_oracle_adjoint,
                test_oracle_postfilter, test_oracle_pbas_gradient, test_oracle_static):
        assert _caught(mod) is None, mod.__name__
