"""GPU parity: the HIP path through the C ABI against the CPU oracle on the same seeded
inputs.  Bar: masks may differ on at most 0.01 % of pixel-frames and float state within
1e-4 relative (|a-b| <= 1e-4 max(|a|,|b|) + 1e-7); PBAS integer state exact.  Both
sides round every operation the same way, so the expected result is bit-exact and the
actual counts are printed."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_gmm_state, compare_pbas_state, log, to_dev  # noqa: E402
from oracle.gmm import GmmParams, GmmRef  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402
from synth import Scene, preset  # noqa: E402

MASK_TOL = 1e-4   # fraction of pixel-frames


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()           # fails loudly if libfgs.so is not built
    yield


def _gmm_params_c(p: GmmParams):
    from paper_2002_00250_amd import fgs
    c = fgs.fgs_gmm_params_default()
    c.Kc, c.Kd = p.Kc, p.Kd
    c.alpha, c.lambda_, c.T_bg, c.w_init = p.alpha, p.lam, p.T_bg, p.w_init
    c.v_init_c, c.v_min_c, c.v_init_d, c.v_min_d = p.v_init_c, p.v_min_c, p.v_init_d, p.v_min_d
    c.w_depth, c.depth_max_mm = p.w_depth, p.depth_max_mm
    c.rho_mode = p.rho_mode
    c.decision, c.density_scale, c.density_threshold = p.decision, p.density_scale, p.density_threshold
    c.var_mode = p.var_mode
    return c


def _pbas_params_c(p: PbasParams):
    from paper_2002_00250_amd import fgs
    c = fgs.fgs_pbas_params_default()
    c.N, c.min_matches = p.N, p.min_matches
    c.R_incdec, c.R_scale, c.T_inc, c.T_dec = p.R_incdec, p.R_scale, p.T_inc, p.T_dec
    c.T_lower, c.T_upper = p.T_lower, p.T_upper
    for j in range(4):
        c.R_lower[j] = p.R_lower[j]
    c.depth_max_mm, c.seed = p.depth_max_mm, p.seed
    c.gradient, c.grad_alpha = int(p.gradient), p.grad_alpha
    return c


def _model(algo, H, W, params):
    from paper_2002_00250_amd import fgs
    cp = _gmm_params_c(params) if algo == fgs.FGS_GMM else _pbas_params_c(params)
    return fgs.Model(algo, H, W, cp)


# ------------------------------------------------------------------ Philox
def test_philox_words_match_oracle():
    from paper_2002_00250_amd import fgs
    from oracle.philox import philox4x32_10
    n = 1 << 20
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4096, 1:] = 0
    ctr[:4096, 0] = np.arange(4096)
    seed = 0x0123456789ABCDEF
    dc = torch.from_numpy(ctr.view(np.int32)).cuda()
    out = torch.zeros_like(dc)
    fgs.fgs_philox4x32_10(seed, dc.data_ptr(), out.data_ptr(), n, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    exp = np.stack(philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], seed & 0xFFFFFFFF, seed >> 32), -1)
    bad = int((got != exp).sum())
    log(f"philox: {n} counters, {bad} words differ")
    assert bad == 0


# ------------------------------------------------------------------ GMM
def _run_gmm_pair(cfg, p, frames, host_frames=False, strided=False):
    from paper_2002_00250_amd import fgs
    sc = Scene(cfg)
    ref = GmmRef(cfg.H, cfg.W, p)
    m = _model(fgs.FGS_GMM, cfg.H, cfg.W, p)
    diff = total = 0
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        exp = ref.step(rgb, D)
        if host_frames:
            m.push(rgb, D)
        elif strided:
            pad_r = torch.zeros((cfg.H, 3 * cfg.W + 13), dtype=torch.uint8, device="cuda")
            pad_d = torch.zeros((cfg.H, cfg.W + 5), dtype=torch.int16, device="cuda")
            r, d = to_dev(rgb, D)
            pad_r[:, :3 * cfg.W] = r.reshape(cfg.H, -1)
            pad_d[:, :cfg.W] = d
            torch.cuda.synchronize()      # filled on torch's stream, read on the model's
            fgs.fgs_push_frame(m.handle, pad_r.data_ptr(), pad_r.stride(0), pad_d.data_ptr(),
                               pad_d.stride(0) * 2, fgs.FGS_MEM_DEVICE)
            torch.cuda.synchronize()
        else:
            r, d = to_dev(rgb, D)
            m.push(r, d)
        got = m.mask_host()
        diff += int((got != exp).sum())
        total += got.size
    n, bad, neq = compare_gmm_state(m.state(), ref.state_planes())
    m.close()
    return diff, total, n, bad, neq


def test_gmm_parity_320x240_k3_100_frames():
    cfg = preset("gmm_320x240")
    diff, total, n, bad, neq = _run_gmm_pair(cfg, GmmParams(Kc=3, Kd=3), 100)
    log(f"gmm 320x240 K=3 100 frames: mask diff {diff}/{total}, state bad {bad}/{n}, not bit-equal {neq}")
    assert diff <= MASK_TOL * total and bad == 0


@pytest.mark.parametrize("H,W,Kc,Kd,frames,mode", [
    (1, 1, 3, 3, 20, "device"),
    (7, 13, 5, 5, 30, "device"),
    (33, 257, 7, 3, 25, "device"),
    (19, 70, 1, 1, 25, "host"),
    (24, 50, 7, 7, 25, "strided"),
    (48, 64, 2, 2, 25, "device"),
    (41, 37, 4, 4, 25, "host"),
    (40, 40, 6, 6, 25, "device"),
])
def test_gmm_parity_edge_shapes(H, W, Kc, Kd, frames, mode):
    cfg = preset("gmm_320x240", H=H, W=W, n_objects=2)
    diff, total, n, bad, neq = _run_gmm_pair(cfg, GmmParams(Kc=Kc, Kd=Kd), frames,
                                             host_frames=mode == "host", strided=mode == "strided")
    log(f"gmm {H}x{W} K={Kc}/{Kd} {mode}: mask diff {diff}/{total}, state bad {bad}, not bit-equal {neq}")
    assert diff == 0 and bad == 0


@pytest.mark.parametrize("Kc,Kd,alpha", [(3, 3, 0.01), (5, 5, 0.05), (7, 3, 0.001)])
def test_gmm_parity_rho_over_w(Kc, Kd, alpha):
    # update-rate variant rho = alpha / w: bit-exact like the default rate
    cfg = preset("gmm_320x240", H=45, W=131, n_objects=3, illumination=True)
    p = GmmParams(Kc=Kc, Kd=Kd, alpha=alpha, rho_mode=1)
    diff, total, n, bad, neq = _run_gmm_pair(cfg, p, 40)
    log(f"gmm rho=alpha/w K={Kc}/{Kd} alpha={alpha}: mask diff {diff}/{total}, state bad {bad}, "
        f"not bit-equal {neq}")
    assert diff == 0 and bad == 0 and neq == 0


@pytest.mark.parametrize("Kc,Kd,rho_mode,tau", [(3, 3, 0, 1.0), (5, 5, 1, 1.0), (7, 3, 0, 50.0)])
def test_gmm_parity_density_decision(Kc, Kd, rho_mode, tau):
    # decision from the scaled Eq. (1) factors: exp is not correctly rounded on either side,
    # so masks may differ where the product sits within an ulp of the threshold (tolerance
    # MASK_TOL); the model state does not depend on the decision and stays bit-exact.
    cfg = preset("gmm_320x240", H=61, W=97, n_objects=3, camouflage=True)
    p = GmmParams(Kc=Kc, Kd=Kd, rho_mode=rho_mode, decision=1, density_threshold=tau)
    diff, total, n, bad, neq = _run_gmm_pair(cfg, p, 40)
    log(f"gmm density decision K={Kc}/{Kd} rho_mode={rho_mode} tau={tau}: mask diff {diff}/{total}, "
        f"state bad {bad}, not bit-equal {neq}")
    assert diff <= MASK_TOL * total and bad == 0 and neq == 0


def test_gmm_parity_rho_alpha_eta():
    # rate alpha * eta (Eq. (1) density): exp differs in the last bit between the oracle
    # and the GPU, so the state agrees to the stated tolerance (1e-4 relative), not bit for bit
    cfg = preset("gmm_320x240", H=45, W=131, n_objects=3, illumination=True)
    p = GmmParams(Kc=5, Kd=5, alpha=0.05, rho_mode=2)
    diff, total, n, bad, neq = _run_gmm_pair(cfg, p, 40)
    log(f"gmm rho=alpha*eta K=5/5: mask diff {diff}/{total}, state bad {bad}/{n}, not bit-equal {neq}")
    assert diff <= MASK_TOL * total and bad == 0


@pytest.mark.parametrize("Kc,Kd,rho_mode,decision,mode", [
    (3, 3, 0, 0, "device"), (5, 5, 1, 0, "host"), (7, 3, 0, 1, "device"), (1, 1, 0, 0, "strided")])
def test_gmm_parity_per_channel_variances(Kc, Kd, rho_mode, decision, mode):
    # one variance per colour channel (v_init and v_min split evenly over the channels):
    # bit-exact model state; masks exact except for the density decision's exp (MASK_TOL)
    cfg = preset("gmm_320x240", H=45, W=131, n_objects=3, illumination=True, camouflage=True)
    p = GmmParams(Kc=Kc, Kd=Kd, rho_mode=rho_mode, decision=decision, var_mode=1)
    diff, total, n, bad, neq = _run_gmm_pair(cfg, p, 40, host_frames=mode == "host",
                                             strided=mode == "strided")
    log(f"gmm per-channel variances K={Kc}/{Kd} rho_mode={rho_mode} decision={decision} {mode}: "
        f"mask diff {diff}/{total}, state bad {bad}/{n}, not bit-equal {neq}")
    assert bad == 0 and neq == 0
    assert diff == 0 if decision == 0 else diff <= MASK_TOL * total


def test_gmm_per_channel_state_round_trip():
    # the exported blob carries the per-channel flag; restoring it into a model with the
    # same parameters continues bit for bit, and both follow the oracle's own run
    from paper_2002_00250_amd import fgs
    cfg = preset("gmm_320x240", H=33, W=71, n_objects=2)
    p = GmmParams(Kc=7, Kd=3, var_mode=1)
    sc = Scene(cfg)
    frames = [sc.frame(t)[:2] for t in range(24)]
    a = _model(fgs.FGS_GMM, cfg.H, cfg.W, p)
    for rgb, D in frames[:12]:
        a.push(*to_dev(rgb, D))
    blob = a.state_blob()
    st = fgs.unpack_state(blob)
    assert st["v_c"].shape == (7, 3, cfg.H, cfg.W)
    np.testing.assert_array_equal(fgs.pack_state(st), blob)
    b = _model(fgs.FGS_GMM, cfg.H, cfg.W, p)
    b.set_state(blob)
    with pytest.raises(fgs.FgsError) as e:          # isotropic model: layout mismatch
        _model(fgs.FGS_GMM, cfg.H, cfg.W, GmmParams(Kc=7, Kd=3)).set_state(blob)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    ref = GmmRef(cfg.H, cfg.W, p)                   # from frame 0, on its own
    for rgb, D in frames[:12]:
        ref.step(rgb, D)
    for rgb, D in frames[12:]:
        a.push(*to_dev(rgb, D))
        b.push(*to_dev(rgb, D))
        exp = ref.step(rgb, D)
        np.testing.assert_array_equal(a.mask_host(), b.mask_host())
        np.testing.assert_array_equal(a.mask_host(), exp)
    np.testing.assert_array_equal(a.state_blob(), b.state_blob())
    n, bad, neq = compare_gmm_state(a.state(), ref.state_planes())
    assert bad == 0 and neq == 0
    a.close()
    b.close()


def test_model_orders_device_tensors_with_torch_stream():
    # frames uploaded asynchronously on torch's stream and pushed at once, masks written into
    # a tensor and read back on torch's stream at once: the binding orders the two streams
    from paper_2002_00250_amd import fgs
    cfg = preset("gmm_320x240", n_objects=3)
    p = GmmParams(Kc=3, Kd=3)
    sc = Scene(cfg)
    ref = GmmRef(cfg.H, cfg.W, p)
    m = _model(fgs.FGS_GMM, cfg.H, cfg.W, p)
    out = torch.empty((cfg.H, cfg.W), dtype=torch.uint8, device="cuda")
    for t in range(25):
        rgb, D, _ = sc.frame(t)
        r = torch.from_numpy(rgb).pin_memory().cuda(non_blocking=True)
        d = torch.from_numpy(D.view(np.int16)).pin_memory().cuda(non_blocking=True)
        m.push(r, d)
        m.mask_into(out)
        got = out.cpu().numpy()
        np.testing.assert_array_equal(got, ref.step(rgb, D), err_msg=f"frame {t}")
        out.fill_(7)                       # torch overwrites it before the next mask lands
    m.close()


def test_gmm_legacy_params_struct_means_rho_alpha():
    # a caller built against the 52-byte fgs_gmm_params (no rho_mode) gets rho = alpha,
    # whatever follows the struct in memory
    from paper_2002_00250_amd import fgs
    cfg = preset("gmm_320x240", H=30, W=50, n_objects=2)
    c = _gmm_params_c(GmmParams())
    c.struct_size = 52
    c.rho_mode = 1                        # beyond the declared size: must be ignored
    sc = Scene(cfg)
    ref = GmmRef(cfg.H, cfg.W, GmmParams())
    m = fgs.Model(fgs.FGS_GMM, cfg.H, cfg.W, c)
    for t in range(20):
        rgb, D, _ = sc.frame(t)
        m.push(rgb, D)
        assert (m.mask_host() == ref.step(rgb, D)).all(), t
    n, bad, neq = compare_gmm_state(m.state(), ref.state_planes())
    m.close()
    assert bad == 0 and neq == 0


def test_gmm_parity_1280x720_k5_sampled_pixels():
    # Full-size launch (the benchmark configuration); every pixel's recursion is
    # independent, so the oracle follows a random sample of pixels one by one.
    from paper_2002_00250_amd import fgs
    cfg = preset("hd_1280x720")
    p = GmmParams(Kc=5, Kd=5)
    sc = Scene(cfg)
    rng = np.random.default_rng(3)
    sel = np.sort(rng.choice(cfg.H * cfg.W, 4096, replace=False))
    ys, xs = sel // cfg.W, sel % cfg.W
    ref = GmmRef(1, sel.size, p)
    m = _model(fgs.FGS_GMM, cfg.H, cfg.W, p)
    diff = total = 0
    frames = 200
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        r, d = to_dev(rgb, D)
        m.push(r, d)
        exp = ref.step(rgb[ys, xs][None], D[ys, xs][None])[0]
        got = m.mask_host()[ys, xs]
        diff += int((got != exp).sum())
        total += sel.size
    st = m.state()
    sub = {k: st[k][..., ys, xs] for k in ("w_c", "mu_c", "v_c", "w_d", "mu_d", "v_d")}
    refst = {k: v[..., 0, :] for k, v in ref.state_planes().items() if k != "t"}
    n, bad, neq = compare_gmm_state(sub, refst)
    log(f"gmm 1280x720 K=5 {frames} frames, {sel.size} sampled px: mask diff {diff}/{total}, "
        f"state bad {bad}/{n}, not bit-equal {neq}")
    m.close()
    assert diff <= MASK_TOL * total and bad == 0


def test_gmm_state_round_trip_and_determinism():
    from paper_2002_00250_amd import fgs
    cfg = preset("gmm_320x240", H=60, W=90)
    p = GmmParams(Kc=3, Kd=3)
    sc = Scene(cfg)
    frames = [sc.frame(t)[:2] for t in range(30)]
    a = _model(fgs.FGS_GMM, 60, 90, p)
    for rgb, D in frames[:15]:
        a.push(*to_dev(rgb, D))
    blob = a.state_blob()
    b = _model(fgs.FGS_GMM, 60, 90, p)
    b.set_state(blob)
    assert b.t == 15
    np.testing.assert_array_equal(b.state_blob(), blob)
    for rgb, D in frames[15:]:
        a.push(*to_dev(rgb, D))
        b.push(*to_dev(rgb, D))
        np.testing.assert_array_equal(a.mask_host(), b.mask_host())
    np.testing.assert_array_equal(a.state_blob(), b.state_blob())
    # the restored run ends where the oracle's own run from frame 0 ends
    ref = GmmRef(60, 90, p)
    for rgb, D in frames:
        ref.step(rgb, D)
    n, bad, neq = compare_gmm_state(b.state(), ref.state_planes())
    assert bad == 0 and neq == 0
    a.close()
    b.close()


# ------------------------------------------------------------------ PBAS
def _run_pbas_pair(cfg, p, frames, host_frames=False):
    from paper_2002_00250_amd import fgs
    sc = Scene(cfg)
    ref = PbasRef(cfg.H, cfg.W, p)
    m = _model(fgs.FGS_PBAS, cfg.H, cfg.W, p)
    diff = total = 0
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        exp = ref.step(rgb, D)
        if host_frames:
            m.push(rgb, D)
        else:
            m.push(*to_dev(rgb, D))
        got = m.mask_host()
        diff += int((got != exp).sum())
        total += got.size
    res = compare_pbas_state(m.state(), ref.state_planes())
    m.close()
    return diff, total, res


@pytest.mark.parametrize("H,W,N,frames,mode", [
    (70, 90, 20, 90, "device"),     # several 64x4 tiles, ragged in x and y
    (1, 1, 2, 20, "device"),
    (5, 3, 4, 30, "host"),
    (9, 130, 8, 40, "device"),
    (37, 64, 35, 70, "device"),
    (21, 70, 41, 60, "device"),     # class 48: last quad not loaded (41 <= 44)
    (21, 70, 47, 65, "host"),       # class 48: last quad loaded, one padding slot
    (13, 67, 53, 70, "device"),     # class 56
    (13, 67, 64, 80, "device"),     # class 64, the largest N
    (6, 40, 3, 25, "device"),       # class 8 with one quad of padding
])
def test_pbas_parity_trajectories(H, W, N, frames, mode):
    cfg = preset("pbas_640x480", H=H, W=W)
    p = PbasParams(N=N, seed=0xABC + N)
    diff, total, res = _run_pbas_pair(cfg, p, frames, host_frames=mode == "host")
    log(f"pbas {H}x{W} N={N} {frames} frames: mask diff {diff}/{total}, state {res}")
    assert diff <= MASK_TOL * total
    assert res["samples"] == 0 and res["dhist"] == 0 and res["S"] == 0
    assert res["R"] == 0 and res["T"] == 0


def test_pbas_state_round_trip_and_determinism():
    from paper_2002_00250_amd import fgs
    cfg = preset("pbas_640x480", H=50, W=70)
    p = PbasParams(N=10)
    sc = Scene(cfg)
    frames = [sc.frame(t)[:2] for t in range(40)]
    a = _model(fgs.FGS_PBAS, 50, 70, p)
    c = _model(fgs.FGS_PBAS, 50, 70, p)
    for rgb, D in frames[:25]:
        a.push(*to_dev(rgb, D))
        c.push(*to_dev(rgb, D))
    blob = a.state_blob()           # applies pending neighbour writes
    b = _model(fgs.FGS_PBAS, 50, 70, p)
    b.set_state(blob)
    for rgb, D in frames[25:]:
        for mdl in (a, b, c):
            mdl.push(*to_dev(rgb, D))
        ma, mb, mc = a.mask_host(), b.mask_host(), c.mask_host()
        np.testing.assert_array_equal(ma, mb)
        np.testing.assert_array_equal(ma, mc)   # reading the state does not perturb the run
    np.testing.assert_array_equal(a.state_blob(), b.state_blob())
    np.testing.assert_array_equal(a.state_blob(), c.state_blob())
    ref = PbasRef(50, 70, p)                          # the oracle's own run from frame 0
    for rgb, D in frames:
        ref.step(rgb, D)
    res = compare_pbas_state(b.state(), ref.state_planes())
    assert all(v == 0 for v in res.values()), res
    for mdl in (a, b, c):
        mdl.close()


# ------------------------------------------------------------------ ABI behaviour
def test_error_paths():
    from paper_2002_00250_amd import fgs
    m = fgs.Model(fgs.FGS_GMM, 8, 8)
    with pytest.raises(fgs.FgsError) as e:
        m.mask_host()
    assert e.value.status == fgs.FGS_ERR_BAD_STATE
    r = torch.zeros((8, 8, 3), dtype=torch.uint8, device="cuda")
    d = torch.zeros((8, 8), dtype=torch.int16, device="cuda")
    with pytest.raises(fgs.FgsError) as e:
        fgs.fgs_push_frame(m.handle, r.data_ptr(), 5, d.data_ptr(), 16, fgs.FGS_MEM_DEVICE)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    m.push(r, d)
    assert m.t == 1 and not m.mask_host().any()
    with pytest.raises(fgs.FgsError):
        m.set_state(np.zeros(10, np.uint8))
    # device state buffers must be 4-byte aligned (checked before any device work)
    size = len(m.state_blob())
    buf = torch.zeros(size + 8, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()      # the fill runs on torch's stream, the copy on the model's
    for call in (lambda: fgs.fgs_copy_state(m.handle, buf.data_ptr() + 2, size, fgs.FGS_MEM_DEVICE),
                 lambda: fgs.fgs_set_state(m.handle, buf.data_ptr() + 1, size, fgs.FGS_MEM_DEVICE)):
        with pytest.raises(fgs.FgsError) as e:
            call()
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    fgs.fgs_copy_state(m.handle, buf.data_ptr() + 4, size, fgs.FGS_MEM_DEVICE)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(buf[4:4 + size].cpu().numpy(), m.state_blob())
    p = fgs.fgs_gmm_params_default()
    p.Kc, p.Kd = 4, 2
    with pytest.raises(fgs.FgsError):
        fgs.Model(fgs.FGS_GMM, 8, 8, p)
    m.close()


def test_copy_probe_copies_and_checks_alignment():
    # the plain streaming copy that calibrates the bandwidth ceiling copies exactly
    from paper_2002_00250_amd import fgs
    n = (1 << 20) + 48
    a = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    b = torch.zeros(n + 32, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    fgs.fgs_copy_probe(a.data_ptr(), b.data_ptr() + 16, n, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(b[16:16 + n], a) and not b[:16].any() and not b[16 + n:].any()
    for src, dst, nb in ((a.data_ptr() + 4, b.data_ptr(), 64), (a.data_ptr(), b.data_ptr() + 8, 64),
                         (a.data_ptr(), b.data_ptr(), 40)):
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_copy_probe(src, dst, nb, torch.cuda.current_stream().cuda_stream)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG
