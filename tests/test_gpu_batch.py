"""Batched pushes (fgs_push_frames): one frame to each of several independent models in
as few launches as their kinds and classes allow.  Every model's masks and state equal the
oracle's own run of that model, bit for bit, through fill frames, mixed sizes, kernel
variants, register classes, groups larger than one launch holds, and GMM and PBAS models
in one call; the argument checks leave every model untouched."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_gmm_state, compare_pbas_state, log, to_dev  # noqa: E402
from oracle.gmm import GmmParams, GmmRef  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402
from synth import Scene, preset  # noqa: E402
from test_gpu_parity import _gmm_params_c, _pbas_params_c  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _run_batched(specs, frames, seed, policy=None):
    """specs: [(algo, H, W, oracle params)]; all models on one stream, pushed together;
    `policy` an fgs_set_cache_policy value for every model (None: the automatic one)."""
    from paper_2002_00250_amd import fgs
    stream = torch.cuda.Stream()
    models, refs, scenes = [], [], []
    for k, (algo, H, W, p) in enumerate(specs):
        cp = _gmm_params_c(p) if algo == fgs.FGS_GMM else _pbas_params_c(p)
        models.append(fgs.Model(algo, H, W, cp, stream=stream))
        if policy is not None:
            fgs.fgs_set_cache_policy(models[-1].handle, policy)
        refs.append(GmmRef(H, W, p) if algo == fgs.FGS_GMM else PbasRef(H, W, p))
        scenes.append(Scene(preset("pbas_640x480", H=H, W=W, seed=seed + k)))
    diff = [0] * len(specs)
    with torch.cuda.stream(stream):
        for t in range(frames):
            rgbs, deps, exps = [], [], []
            for sc, ref in zip(scenes, refs):
                rgb, D, _ = sc.frame(t)
                exps.append(ref.step(rgb, D))
                r, d = to_dev(rgb, D)
                rgbs.append(r)
                deps.append(d)
            fgs.push_frames(models, rgbs, deps)
            for k, (m, e) in enumerate(zip(models, exps)):
                diff[k] += int((m.mask_host() != e).sum())
    out = []
    for (algo, H, W, p), m, ref, dk in zip(specs, models, refs, diff):
        if algo == fgs.FGS_GMM:
            n, bad, neq = compare_gmm_state(m.state(), ref.state_planes())
            out.append(("gmm", H, W, dk, {"bad": bad, "not_bit_equal": neq}))
        else:
            out.append(("pbas", H, W, dk, compare_pbas_state(m.state(), ref.state_planes())))
        m.close()
    return out


def _all_equal(res):
    for kind, H, W, dk, st in res:
        log(f"batched {kind} {H}x{W}: mask diff {dk}, state {st}")
        assert dk == 0 and all(v == 0 for v in st.values()), (kind, H, W, dk, st)


def test_gmm_models_of_several_sizes_and_variants():
    from paper_2002_00250_amd import fgs
    G = fgs.FGS_GMM
    specs = [(G, 48, 80, GmmParams(Kc=5, Kd=5)), (G, 37, 129, GmmParams(Kc=5, Kd=5)),
             (G, 64, 64, GmmParams(Kc=5, Kd=5)), (G, 40, 50, GmmParams(Kc=7, Kd=3)),
             (G, 33, 70, GmmParams(Kc=5, Kd=5, rho_mode=1)), (G, 20, 300, GmmParams(Kc=3, Kd=3)),
             (G, 1, 257, GmmParams(Kc=5, Kd=5))]
    _all_equal(_run_batched(specs, 14, seed=11))


def test_more_models_than_one_launch_holds():
    from paper_2002_00250_amd import fgs
    specs = [(fgs.FGS_GMM, 24 + k, 40 + 3 * k, GmmParams(Kc=3, Kd=3)) for k in range(11)]
    _all_equal(_run_batched(specs, 8, seed=40))


def test_pbas_models_through_fill_frames_and_classes():
    # N = 35 keeps the previous value in a padding slot, N = 36 does not; N = 33 shares
    # their register class; N = 5 and 20 are classes of their own; the fill frames of the
    # smaller N end first, so fill launches and batched steps mix in one call
    from paper_2002_00250_amd import fgs
    P = fgs.FGS_PBAS
    specs = [(P, 21, 70, PbasParams(N=35, seed=1)), (P, 9, 130, PbasParams(N=36, seed=2)),
             (P, 16, 64, PbasParams(N=33, seed=3)), (P, 13, 40, PbasParams(N=5, seed=4)),
             (P, 30, 66, PbasParams(N=20, seed=5)), (P, 4, 64, PbasParams(N=35, seed=6))]
    _all_equal(_run_batched(specs, 44, seed=60))


def test_gmm_and_pbas_in_one_call():
    from paper_2002_00250_amd import fgs
    specs = [(fgs.FGS_PBAS, 20, 70, PbasParams(N=6, seed=9)), (fgs.FGS_GMM, 20, 70, GmmParams(Kc=5, Kd=5)),
             (fgs.FGS_PBAS, 17, 90, PbasParams(N=6, seed=10)), (fgs.FGS_GMM, 31, 33, GmmParams(Kc=5, Kd=5))]
    _all_equal(_run_batched(specs, 12, seed=80))


def test_benchmark_kernel_instances_on_distinct_models():
    # The instances the benchmark times: 8 GMM Kc = Kd = 5 models (default rate and
    # decision) in one launch and 4 PBAS N = 35 models in one launch, state streamed with
    # non-temporal accesses.  Small ragged frames, every model its own scene and seed, so a
    # workgroup that took another model's arguments would show.
    from paper_2002_00250_amd import fgs
    G, P = fgs.FGS_GMM, fgs.FGS_PBAS
    sizes = [(37, 129), (48, 80), (1, 257), (64, 64), (33, 70), (20, 300), (45, 131), (17, 95)]
    specs = [(G, H, W, GmmParams(Kc=5, Kd=5)) for H, W in sizes]
    specs += [(P, H, W, PbasParams(N=35, seed=100 + k))
              for k, (H, W) in enumerate([(21, 70), (45, 131), (9, 130), (64, 66)])]
    _all_equal(_run_batched(specs, 50, seed=120, policy=fgs.FGS_CACHE_STREAM))


def test_kinds_on_two_streams_overlapping():
    # The benchmark's --kind-streams mode: the 8-model GMM launch on one stream and the
    # 4-model PBAS launch on another, issued back to back with the raw batch call (no
    # stream waits between them), so the two kinds run at the same time on the device.
    # Every model still equals its oracle run.
    from paper_2002_00250_amd import fgs
    G, P = fgs.FGS_GMM, fgs.FGS_PBAS
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    gsizes = [(37, 129), (48, 80), (1, 257), (64, 64), (33, 70), (20, 300), (45, 131), (17, 95)]
    psizes = [(21, 70), (45, 131), (9, 130), (64, 66)]
    specs = [(G, H, W, GmmParams(Kc=5, Kd=5), sa) for H, W in gsizes]
    specs += [(P, H, W, PbasParams(N=35, seed=200 + k), sb) for k, (H, W) in enumerate(psizes)]
    frames = 45
    models, refs, inputs = [], [], []
    for k, (algo, H, W, p, st) in enumerate(specs):
        cp = _gmm_params_c(p) if algo == G else _pbas_params_c(p)
        m = fgs.Model(algo, H, W, cp, stream=st)
        fgs.fgs_set_cache_policy(m.handle, fgs.FGS_CACHE_STREAM)
        models.append(m)
        refs.append(GmmRef(H, W, p) if algo == G else PbasRef(H, W, p))
        sc = Scene(preset("pbas_640x480", H=H, W=W, seed=300 + k))
        inputs.append([sc.frame(t)[:2] for t in range(frames)])
    dev = [[to_dev(rgb, D) for rgb, D in fr] for fr in inputs]
    torch.cuda.synchronize()      # every frame resident before the first launch
    kinds = [[k for k, sp in enumerate(specs) if sp[0] == a] for a in (G, P)]
    diff = [0] * len(specs)
    for t in range(frames):
        for ks in kinds:
            fgs.fgs_push_frames([models[k].handle for k in ks], [dev[k][t][0].data_ptr() for k in ks],
                                [dev[k][t][0].stride(0) for k in ks], [dev[k][t][1].data_ptr() for k in ks],
                                [2 * dev[k][t][1].stride(0) for k in ks])
        for k, (m, ref) in enumerate(zip(models, refs)):
            e = ref.step(*inputs[k][t])
            diff[k] += int((m.mask_host() != e).sum())
    res = []
    for (algo, H, W, _, _), m, ref, dk in zip(specs, models, refs, diff):
        if algo == G:
            n, bad, neq = compare_gmm_state(m.state(), ref.state_planes())
            res.append(("gmm", H, W, dk, {"bad": bad, "not_bit_equal": neq}))
        else:
            res.append(("pbas", H, W, dk, compare_pbas_state(m.state(), ref.state_planes())))
        m.close()
    _all_equal(res)


def test_argument_checks_leave_models_untouched():
    from paper_2002_00250_amd import fgs
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    gp = fgs.fgs_gmm_params_default()
    a = fgs.Model(fgs.FGS_GMM, 16, 32, gp, stream=s1)
    b = fgs.Model(fgs.FGS_GMM, 16, 32, gp, stream=s1)
    c = fgs.Model(fgs.FGS_GMM, 16, 32, gp, stream=s2)
    rgb = torch.zeros((16, 32, 3), dtype=torch.uint8, device="cuda")
    dep = torch.zeros((16, 32), dtype=torch.int16, device="cuda")
    torch.cuda.synchronize()
    H = lambda ms: [m.handle for m in ms]
    cases = [
        (H([a, b, a]), [rgb.data_ptr()] * 3, [96] * 3, [dep.data_ptr()] * 3, [64] * 3),   # repeated model
        (H([a, c]), [rgb.data_ptr()] * 2, [96] * 2, [dep.data_ptr()] * 2, [64] * 2),      # two streams
        (H([a, b]), [rgb.data_ptr()] * 2, [95, 96], [dep.data_ptr()] * 2, [64] * 2),      # short rgb rows
        (H([a, b]), [rgb.data_ptr()] * 2, [96] * 2, [dep.data_ptr()] * 2, [64, 63]),      # odd depth stride
        (H([a, b]), [rgb.data_ptr(), 0], [96] * 2, [dep.data_ptr()] * 2, [64] * 2),       # NULL frame
        ([], [], [], [], []),                                                              # n = 0
    ]
    for args in cases:
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_push_frames(*args)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG, args
    assert a.t == b.t == c.t == 0
    with pytest.raises(ValueError):
        fgs.push_frames([a, b], [rgb, rgb[:8]], [dep, dep])                                # wrong size
    fgs.push_frames([a, b], [rgb, rgb], [dep, dep])
    assert a.t == b.t == 1 and c.t == 0
    for m in (a, b, c):
        m.close()
