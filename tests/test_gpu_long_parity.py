"""Long GPU parity: two workloads followed from frame 0 over their whole length, every
mask and the final state compared with the oracle's own run (no restart from the GPU's
state anywhere).

* PBAS N = 20 at 640x480 over 300 frames (illumination ramp, colour-camouflaged object):
  one model, the whole image against one oracle run.
* The benchmark's workload in its launch configuration over a 200-frame prefix of the
  1280x720 sequence (8 objects, shadows): 8 GMM Kc = Kd = 5 models and 4 PBAS N = 35
  models on one stream, one fgs_push_frames call per kind and frame, so the eight-model
  GMM and PBAS kernel instances run, streaming their state (2.4 GB live, beyond the
  last-level cache).  The models of a kind see the same frames: each must equal the
  others and the oracle.  GMM is compared with 8 row bands of the image (each pixel's
  mixture is its own, so a band is exact); PBAS with 2 x 4 windows widened by the
  propagation margin of the neighbour updates (165 pixels after 165 updating frames),
  each owning a rectangle of the image.

The oracle runs in child processes (tests/oracle_runs.py) while this process drives the
GPU.  Bar as in test_gpu_parity.py; the expected counts are zero and are printed."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_gmm_state, compare_pbas_state, log, to_dev  # noqa: E402
from oracle.gmm import GmmParams  # noqa: E402
from oracle.pbas import PbasParams  # noqa: E402
from oracle_runs import OracleRuns, make_job, windows  # noqa: E402
from synth import Scene, preset  # noqa: E402
from test_gpu_parity import MASK_TOL, _gmm_params_c, _pbas_params_c  # noqa: E402

VGA_FRAMES, VGA_N = 300, 20
HD_FRAMES, HD_K, HD_N, HD_G, HD_P = 200, 5, 35, 8, 4
HD_GMM_BANDS = 8
HD_PBAS_GRID = (2, 4)


@pytest.fixture(scope="module")
def oracle(tmp_path_factory):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    jobs, idx = [], {"vga": [], "gmm": [], "pbas": []}
    H, W = 480, 640
    for win, own in windows(H, W, 1, 1, 0):
        idx["vga"].append(len(jobs))
        jobs.append(make_job("pbas", "pbas_640x480", {}, dict(N=VGA_N), VGA_FRAMES, H, W, win, own))
    H, W = 720, 1280
    for win, own in windows(H, W, *HD_PBAS_GRID, HD_FRAMES - HD_N):
        idx["pbas"].append(len(jobs))
        jobs.append(make_job("pbas", "hd_1280x720", {}, dict(N=HD_N), HD_FRAMES, H, W, win, own))
    for win, own in windows(H, W, HD_GMM_BANDS, 1, 0):
        idx["gmm"].append(len(jobs))
        jobs.append(make_job("gmm", "hd_1280x720", {}, dict(Kc=HD_K, Kd=HD_K), HD_FRAMES, H, W, win, own))
    runs = OracleRuns(jobs, str(tmp_path_factory.mktemp("oracle_runs")))
    log(f"long parity: {len(jobs)} oracle jobs started")
    yield runs, idx
    runs.close()


def _assemble(runs, ids, H, W, frames):
    """Masks [frames, H, W] (bool) and the final state planes over the whole image."""
    masks = np.zeros((frames, H, W), bool)
    state = {}
    for i in ids:
        oy, ox, oh, ow = runs.jobs[i]["own"]
        res = runs.result(i)
        m = np.unpackbits(res["masks"], axis=1)[:, :oh * ow].reshape(frames, oh, ow)
        masks[:, oy:oy + oh, ox:ox + ow] = m.astype(bool)
        for k, v in res.items():
            if k.startswith("state_"):
                k = k[len("state_"):]
                if k not in state:
                    state[k] = np.zeros(v.shape[:-2] + (H, W), v.dtype)
                state[k][..., oy:oy + oh, ox:ox + ow] = v
    return masks, state


def _mask_diffs(got_packed, exp, H, W):
    per = []
    for t in range(exp.shape[0]):
        g = np.unpackbits(got_packed[t])[:H * W].reshape(H, W).astype(bool)
        per.append(int((g != exp[t]).sum()))
    return per


def test_pbas_640x480_n20_all_300_frames(oracle):
    from paper_2002_00250_amd import fgs
    runs, idx = oracle
    cfg = preset("pbas_640x480")
    H, W = cfg.H, cfg.W
    p = PbasParams(N=VGA_N)
    sc = Scene(cfg)
    m = fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p))
    got = []
    for t in range(VGA_FRAMES):
        rgb, D, _ = sc.frame(t)
        m.push(*to_dev(rgb, D))
        mk = m.mask_host()
        assert np.isin(mk, (0, 255)).all()
        got.append(np.packbits(mk != 0))
    st = m.state()
    m.close()
    exp, exp_state = _assemble(runs, idx["vga"], H, W, VGA_FRAMES)
    per = _mask_diffs(got, exp, H, W)
    res = compare_pbas_state(st, exp_state)
    fg = int(exp.sum())
    log(f"pbas 640x480 N=20 {VGA_FRAMES} frames from frame 0: mask diff {sum(per)}/{VGA_FRAMES * H * W} "
        f"(worst frame {max(per)}; {fg} foreground pixel-frames), final state {res}")
    assert sum(per) <= MASK_TOL * VGA_FRAMES * H * W
    assert all(v == 0 for v in res.values()), res


def test_benchmark_workload_1280x720_200_frames(oracle):
    from paper_2002_00250_amd import fgs
    runs, idx = oracle
    cfg = preset("hd_1280x720")
    H, W = cfg.H, cfg.W
    sc = Scene(cfg)
    stream = torch.cuda.Stream()
    gp = _gmm_params_c(GmmParams(Kc=HD_K, Kd=HD_K))
    pp = _pbas_params_c(PbasParams(N=HD_N))
    gms = [fgs.Model(fgs.FGS_GMM, H, W, gp, stream=stream) for _ in range(HD_G)]
    pms = [fgs.Model(fgs.FGS_PBAS, H, W, pp, stream=stream) for _ in range(HD_P)]
    live = sum(fgs.fgs_device_bytes(m.handle) for m in gms + pms)
    thr = int(os.environ.get("FGS_STREAMING_THRESHOLD_MB", "192")) << 20
    log(f"benchmark workload: {HD_G} GMM + {HD_P} PBAS models, {live / 2**30:.2f} GiB live "
        f"(streaming above {thr >> 20} MiB)")
    assert live > thr                         # the automatic policy streams, as in the benchmark
    outs = {k: torch.empty((len(ms), H, W), dtype=torch.uint8, device="cuda")
            for k, ms in (("gmm", gms), ("pbas", pms))}
    got = {"gmm": [], "pbas": []}
    twins = {"gmm": 0, "pbas": 0}
    with torch.cuda.stream(stream):
        for t in range(HD_FRAMES):
            rgb, D, _ = sc.frame(t)
            r, d = to_dev(rgb, D)
            for kind, ms in (("gmm", gms), ("pbas", pms)):
                fgs.push_frames(ms, [r] * len(ms), [d] * len(ms))
            for kind, ms in (("gmm", gms), ("pbas", pms)):
                o = outs[kind]
                for j, mdl in enumerate(ms):
                    mdl.mask_into(o[j])
                twins[kind] += int((o[1:] != o[:1]).sum().item())
                got[kind].append(np.packbits(o[0].cpu().numpy() != 0))
    torch.cuda.synchronize()
    blobs_equal = {}
    for kind, ms in (("gmm", gms), ("pbas", pms)):
        b0 = ms[0].state_blob()
        blobs_equal[kind] = all(np.array_equal(b0, mdl.state_blob()) for mdl in ms[1:])
        del b0
    gst, pst = gms[0].state(), pms[0].state()
    for mdl in gms + pms:
        mdl.close()
    log(f"benchmark workload: models of a kind equal each other: masks {twins}, state {blobs_equal}")
    assert twins == {"gmm": 0, "pbas": 0} and all(blobs_equal.values())

    exp, exp_state = _assemble(runs, idx["gmm"], H, W, HD_FRAMES)
    per = _mask_diffs(got["gmm"], exp, H, W)
    n, bad, neq = compare_gmm_state(gst, exp_state)
    log(f"gmm 1280x720 K=5 in the 8-model streaming launch, {HD_FRAMES} frames: mask diff "
        f"{sum(per)}/{HD_FRAMES * H * W}, state bad {bad}/{n}, not bit-equal {neq}")
    assert sum(per) <= MASK_TOL * HD_FRAMES * H * W and bad == 0
    del exp, exp_state, gst

    exp, exp_state = _assemble(runs, idx["pbas"], H, W, HD_FRAMES)
    per = _mask_diffs(got["pbas"], exp, H, W)
    res = compare_pbas_state(pst, exp_state)
    log(f"pbas 1280x720 N=35 in the 8-model streaming launch, {HD_FRAMES} frames (windows with a "
        f"{HD_FRAMES - HD_N}-pixel margin): mask diff {sum(per)}/{HD_FRAMES * H * W}, final state {res}")
    assert sum(per) <= MASK_TOL * HD_FRAMES * H * W
    assert all(v == 0 for v in res.values()), res
