"""Pins for the PBAS oracle (Sec. 3.2 and the base PBAS rules it adapts).

Checked against: hand-derived frames (tests/golden), invariants of the model (bounds of
R and T, S = sum of D, sample provenance), the update decisions against the Philox words
(pinned separately against the ROCm library), update statistics, and scenes whose
answer is known (static scene, colour camouflage)."""
import json
import os

import numpy as np
import pytest

from oracle.depth import depth_q8
from oracle.pbas import NB_DX, NB_DY, PbasParams, PbasRef, pbas_draws
from synth import Scene, preset

GOLD = os.path.join(os.path.dirname(__file__), "golden", "pbas_hand_cases.json")


def test_hand_derived_frames():
    gold = json.load(open(GOLD))
    pr = dict(gold["params"])
    pr["R_lower"] = tuple(pr["R_lower"])
    for seed in (1, 2, 3, 0xDEADBEEF):       # the answer must not depend on the draws
        ref = PbasRef(1, 1, PbasParams(seed=seed, **pr))
        for fr in gold["frames"]:
            m = ref.step(np.array(fr["rgb"], np.uint8).reshape(1, 1, 3),
                         np.array([[fr["D"]]], np.uint16))
            assert m[0, 0] == fr["mask"], fr["note"]
            if "expect_samples" in fr:
                for j in range(4):
                    assert sorted(ref.samples[:, 0, 0, j].tolist()) == fr["expect_samples"][j], fr["note"]
                    assert sorted(ref.D[:, 0, 0, j].tolist()) == fr["expect_dhist"][j], fr["note"]
                assert ref.S[0, 0].tolist() == fr["expect_S"]
                assert ref.R[0, 0].tolist() == [np.float32(v) for v in fr["expect_R"]]
                assert ref.T[0, 0].tolist() == fr["expect_T"]


def test_hand_derived_boundaries():
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pbas_hand_boundaries.json")))
    pr = dict(gold["params"])
    pr["R_lower"] = tuple(pr["R_lower"])
    for case in gold["cases"]:
        for seed in (1, 7):
            ref = PbasRef(1, 1, PbasParams(seed=seed, **pr))
            for fr in case["fill"]:
                ref.step(np.array(fr["rgb"], np.uint8).reshape(1, 1, 3), np.array([[fr["D"]]], np.uint16))
            fr = case["frame"]
            m = ref.step(np.array(fr["rgb"], np.uint8).reshape(1, 1, 3), np.array([[fr["D"]]], np.uint16))
            assert m[0, 0] == case["mask"], case["note"]


def test_rate_T_rises_for_foreground_and_falls_for_background():
    # the update period T grows where a channel is foreground and shrinks where it is
    # background (clamped to its bounds); channels not processed keep it
    cfg = preset("pbas_640x480", H=48, W=64, n_objects=2)
    p = PbasParams(N=8)
    sc = Scene(cfg)
    ref = PbasRef(48, 64, p)
    up = down = 0
    for t in range(40):
        rgb, D, _ = sc.frame(t)
        T0 = ref.T.copy()
        ref.step(rgb, D)
        if t < p.N:
            continue
        F = ref.last_F
        active = np.ones_like(F)
        active[..., 3] = D > 0
        assert np.all(ref.T[F] >= T0[F]) and np.all(ref.T[active & ~F] <= T0[active & ~F])
        np.testing.assert_array_equal(ref.T[~active], T0[~active])
        up += int((ref.T[F] > T0[F]).sum())
        down += int((ref.T[active & ~F] < T0[active & ~F]).sum())
    assert up > 0 and down > 0


def _run(cfg, params, frames, audit=None):
    sc = Scene(cfg)
    ref = PbasRef(cfg.H, cfg.W, params)
    masks = []
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        before = (ref.T.copy(), ref.samples.copy(), ref.D.copy())
        masks.append(ref.step(rgb, D))
        if audit is not None:
            audit(ref, t, rgb, D, before)
    return ref, masks


def test_invariants_and_provenance():
    cfg = preset("pbas_640x480", H=18, W=22)
    p = PbasParams(N=8)
    seen = np.zeros((256, 18, 22, 4), bool)      # values observed per pixel and channel
    seen[0, :, :, 3] = True                      # depth byte 0 = "no depth recorded"

    def audit(ref, t, rgb, D, before):
        I = ref.frame_value(rgb, D)
        yy, xx = np.mgrid[0:18, 0:22]
        for j in range(4):
            seen[I[..., j], yy, xx, j] = True
        # every sample byte at a pixel is a value that pixel has shown (never a neighbour's)
        for k in range(min(p.N, t + 1)):          # slots >= t+1 are still empty in init
            for j in range(4):
                assert seen[ref.samples[k, :, :, j], yy, xx, j].all(), (t, k, j)
        assert np.all(ref.R >= np.array(p.R_lower, np.float32))
        assert np.all((ref.T >= p.T_lower) & (ref.T <= p.T_upper))
        np.testing.assert_array_equal(ref.S, ref.D.astype(np.int64).sum(0))

    _run(cfg, p, 70, audit)


def test_update_decisions_follow_draws():
    cfg = preset("pbas_640x480", H=10, W=12)
    p = PbasParams(N=6, seed=77)

    def audit(ref, t, rgb, D, before):
        if t < p.N:
            return
        T_prev, samp_prev, D_prev = before
        w0, w1 = pbas_draws(10, 12, t, p.seed)
        u0 = (w0 >> 16).astype(np.float64) / 65536.0
        u1 = (w1 >> 16).astype(np.float64) / 65536.0
        active = np.ones((10, 12, 4), bool)
        active[..., 3] = D > 0
        bg = active & ~ref.last_F
        # the decision uses the rate T from before this frame
        np.testing.assert_array_equal(ref.last_self, bg & (u0 * T_prev.astype(np.float64) < 1.0))
        np.testing.assert_array_equal(ref.last_nb, bg & (u1 * T_prev.astype(np.float64) < 1.0))
        I = ref.frame_value(rgb, D)
        k = ((w0 & 0xFFFF).astype(np.int64) * p.N) >> 16
        ys, xs, js = np.nonzero(ref.last_self)
        assert np.all(ref.samples[k[ys, xs, js], ys, xs, js] == I[ys, xs, js])
        # a pixel's D history changes only in the slot its own self-update chose
        changed = ref.D != D_prev
        n, ys, xs, js = np.nonzero(changed)
        assert np.all(ref.last_self[ys, xs, js]) and np.all(k[ys, xs, js] == n)

    _run(cfg, p, 40, audit)


def test_neighbour_writes_gathered_independently():
    # Recompute frame t's neighbour writes as a gather (each pixel collects the writes
    # aimed at it) and compare with the oracle's scatter.
    cfg = preset("pbas_640x480", H=9, W=11, n_objects=1)
    p = PbasParams(N=5, T_lower=1.0, T_upper=3.0, seed=5)
    sc = Scene(cfg)
    ref = PbasRef(9, 11, p)
    for t in range(30):
        rgb, D, _ = sc.frame(t)
        prev = ref.samples.copy()
        ref.step(rgb, D)
        if t < p.N:
            continue
        I = ref.frame_value(rgb, D)
        w0, w1 = ref.last_draws
        expect = prev.copy()
        k0 = ((w0 & 0xFFFF).astype(np.int64) * p.N) >> 16
        ys, xs, js = np.nonzero(ref.last_self)
        expect[k0[ys, xs, js], ys, xs, js] = I[ys, xs, js]
        direc = (w1 >> 13) & 7
        k1 = ((w1 & 0x1FFF).astype(np.int64) * p.N) >> 13
        for y in range(9):
            for x in range(11):
                for oy in (-1, 0, 1):
                    for ox in (-1, 0, 1):
                        sy, sx = y + oy, x + ox               # a possible source
                        if (ox, oy) == (0, 0) or not (0 <= sy < 9 and 0 <= sx < 11):
                            continue
                        for j in range(4):
                            if not ref.last_nb[sy, sx, j]:
                                continue
                            d = direc[sy, sx, j]
                            if (sx + NB_DX[d], sy + NB_DY[d]) != (x, y):
                                continue
                            if j == 3 and D[y, x] == 0:
                                continue
                            expect[k1[sy, sx, j], y, x, j] = I[y, x, j]
        np.testing.assert_array_equal(ref.samples, expect, err_msg=f"frame {t}")


def test_draws_follow_the_counter_definition():
    # R-17 written out for single pixels: block c of pixel (y, x) at frame t is
    # Philox4x32-10 of the counter (y * W_img + x, t, c, 0) under the key (low 32 bits of
    # the seed, high 32 bits), computed by the one-counter integer implementation with
    # the key split by hand; block 0 serves the self-update, block 1 the neighbour
    # update, word j channel j.  A seed whose halves differ, frames that differ from the
    # block index, and windows placed in a wider image.
    from oracle.philox import philox4x32_10_int
    seed = 0x0123456789ABCDEF
    key = (0x89ABCDEF, 0x01234567)
    cases = [  # (H, W, t, origin or None, pixels (y, x) of the array)
        (5, 7, 3, None, [(0, 0), (0, 6), (4, 0), (2, 3), (4, 6)]),
        (3, 4, 12345, None, [(0, 1), (2, 3)]),
        (4, 5, 2, (10, 20, 640), [(0, 0), (3, 4), (1, 2)]),
        (2, 3, 0xFFFFFFF0, (479, 637, 640), [(0, 0), (1, 2)]),
    ]
    for H, W, t, origin, pts in cases:
        w0, w1 = pbas_draws(H, W, t, seed, origin)
        assert w0.shape == w1.shape == (H, W, 4) and w0.dtype == w1.dtype == np.uint32
        y0, x0, W_img = origin if origin is not None else (0, 0, W)
        for y, x in pts:
            pix = (y0 + y) * W_img + (x0 + x)
            for c, blk in ((0, w0), (1, w1)):
                want = philox4x32_10_int((pix, t, c, 0), key)
                assert tuple(int(v) for v in blk[y, x]) == want, (H, W, t, origin, y, x, c)
    # the two blocks of a pixel-frame are different words (a self-update and a neighbour
    # update drawn from one block would make this fail only by chance)
    w0, w1 = pbas_draws(4, 4, 7, seed)
    assert not np.array_equal(w0, w1)


def test_window_model_matches_whole_image_except_ring_samples():
    # A window of a larger image drawn with the image's pixel indices: from the same state,
    # one frame gives the whole image's mask, R, T, S and D on the window, and its samples
    # everywhere but the window's outermost ring (writes from outside are not modelled).
    cfg = preset("pbas_640x480", H=14, W=18, n_objects=2)
    p = PbasParams(N=6, T_lower=1.0, T_upper=4.0, seed=9)
    sc = Scene(cfg)
    full = PbasRef(14, 18, p)
    y0, x0, h, w = 3, 4, 7, 9
    ring_diff = 0
    w0f, w1f = pbas_draws(14, 18, 11, p.seed)
    w0w, w1w = pbas_draws(h, w, 11, p.seed, (y0, x0, 18))
    np.testing.assert_array_equal(w0w, w0f[y0:y0 + h, x0:x0 + w])
    np.testing.assert_array_equal(w1w, w1f[y0:y0 + h, x0:x0 + w])
    for t in range(24):
        rgb, D, _ = sc.frame(t)
        win = PbasRef(h, w, p, origin=(y0, x0, 18))
        st = full.state_planes()
        win.set_state_planes({k: (v[..., y0:y0 + h, x0:x0 + w] if k != "t" else v) for k, v in st.items()})
        m_win = win.step(rgb[y0:y0 + h, x0:x0 + w], D[y0:y0 + h, x0:x0 + w])
        m_full = full.step(rgb, D)
        np.testing.assert_array_equal(m_win, m_full[y0:y0 + h, x0:x0 + w])
        a, b = win.state_planes(), full.state_planes()
        for k in ("dhist", "R", "T", "S"):
            np.testing.assert_array_equal(a[k], b[k][..., y0:y0 + h, x0:x0 + w], err_msg=f"{k} t={t}")
        sa, sb = a["samples"], b["samples"][:, y0:y0 + h, x0:x0 + w]
        np.testing.assert_array_equal(sa[:, 1:-1, 1:-1], sb[:, 1:-1, 1:-1], err_msg=f"t={t}")
        ring_diff += int((sa != sb).sum())
    assert ring_diff > 0          # writes from outside the window do reach its ring


def test_window_from_frame_zero_matches_inside_a_margin():
    # Run alone from frame 0, a window differs from the whole image only through the writes
    # its outside neighbours send in; after u updating frames every field agrees at least
    # u pixels from the window's inner edges (and the ring does differ at some point).
    cfg = preset("pbas_640x480", H=26, W=34, n_objects=2)
    p = PbasParams(N=4, T_lower=1.0, T_upper=4.0, seed=21)
    sc = Scene(cfg)
    full = PbasRef(26, 34, p)
    y0, x0, h, w = 4, 5, 18, 22
    win = PbasRef(h, w, p, origin=(y0, x0, 34))
    outer_diff = 0
    for t in range(12):
        rgb, D, _ = sc.frame(t)
        mw = win.step(rgb[y0:y0 + h, x0:x0 + w], D[y0:y0 + h, x0:x0 + w])
        mf = full.step(rgb, D)[y0:y0 + h, x0:x0 + w]
        u = max(0, t - p.N + 1)
        inner = (slice(u, h - u), slice(u, w - u))
        a, b = win.state_planes(), full.state_planes()
        np.testing.assert_array_equal(mw[inner], mf[inner], err_msg=f"mask t={t}")
        for k in ("samples", "dhist", "R", "T", "S"):
            bk = b[k][..., y0:y0 + h, x0:x0 + w]
            np.testing.assert_array_equal(a[k][(Ellipsis,) + inner], bk[(Ellipsis,) + inner], err_msg=f"{k} t={t}")
            outer_diff += int((a[k] != bk).sum())
    assert outer_diff > 0


def test_update_rate_and_uniform_choices():
    # Fixed T: the self-update fires with probability 1/T; slots and directions uniform.
    cfg = preset("pbas_640x480", H=64, W=64, n_objects=0, illumination=False, camouflage=False)
    T0 = 4.0
    p = PbasParams(N=16, T_lower=T0, T_upper=T0, seed=123)
    sc = Scene(cfg)
    ref = PbasRef(64, 64, p)
    fires = trials = 0
    slots = np.zeros(p.N, np.int64)
    dirs = np.zeros(8, np.int64)
    for t in range(40):
        ref.step(*sc.frame(t)[:2])
        if t < p.N:
            continue
        bg = ~ref.last_F & np.ones_like(ref.last_F)
        bg[..., 3] &= sc.frame(t)[1] > 0
        trials += int(bg.sum())
        fires += int(ref.last_self.sum())
        w0, w1 = ref.last_draws
        slots += np.bincount((((w0 & 0xFFFF).astype(np.int64) * p.N) >> 16)[ref.last_self], minlength=p.N)
        dirs += np.bincount(((w1 >> 13) & 7)[ref.last_nb].astype(np.int64), minlength=8)
    rate = fires / trials
    sd = np.sqrt(0.25 * 0.75 / trials)
    assert abs(rate - 1 / T0) < 5 * sd
    for c in (slots, dirs):
        e = c.sum() / len(c)
        assert ((c - e) ** 2 / e).sum() < 3 * len(c) + 30


def test_static_noise_free_scene_gives_empty_mask():
    cfg = preset("pbas_640x480", H=16, W=20, n_objects=0, illumination=False, camouflage=False,
                 rgb_noise=0.0, depth_noise_mm=0.0, hole_frac=0.0)
    p = PbasParams(N=6)
    _, masks = _run(cfg, p, 25)
    assert not any(m.any() for m in masks)


def test_colour_camouflage_detected_only_with_depth():
    H, W = 24, 24
    rng = np.random.default_rng(9)
    bg = rng.integers(40, 220, (H, W, 3)).astype(np.uint8)
    D = np.full((H, W), 3000, np.uint16)
    obj = np.zeros((H, W), bool)
    obj[6:16, 8:18] = True
    out = {}
    for use_depth in (True, False):
        ref = PbasRef(H, W, PbasParams(N=10))
        Dm = D if use_depth else np.zeros_like(D)
        for t in range(20):
            ref.step(bg, Dm)
        D2 = D.copy()
        D2[obj] = 2400                      # 600 mm nearer, colour unchanged
        out[use_depth] = ref.step(bg, D2 if use_depth else np.zeros_like(D2))
    assert np.all(out[True][obj] == 255) and not out[True][~obj].any()
    assert not out[False].any()


def test_invalid_depth_pixel_skips_depth_channel():
    cfg = preset("pbas_640x480", H=8, W=8, n_objects=0, illumination=False, camouflage=False)
    p = PbasParams(N=4, T_lower=1.0, T_upper=1.0)
    sc = Scene(cfg)
    ref = PbasRef(8, 8, p)
    for t in range(8):
        ref.step(*sc.frame(t)[:2])
    rgb, D, _ = sc.frame(8)
    D[:] = 0
    before = (ref.samples[..., 3].copy(), ref.D[..., 3].copy(), ref.R[..., 3].copy(), ref.T[..., 3].copy())
    ref.step(rgb, D)
    after = (ref.samples[..., 3], ref.D[..., 3], ref.R[..., 3], ref.T[..., 3])
    for b, a in zip(before, after):
        np.testing.assert_array_equal(a, b)
    assert not ref.last_F[..., 3].any()
