"""The windowed oracle runs used by the long GPU parity tests reassemble the whole-image
oracle exactly: owned rectangles partition the image, and masks and final state taken
from each window's own rectangle equal the whole image's model, for PBAS with the
propagation margin (Sec. 3.2 neighbour updates) and for GMM bands (no margin)."""
import numpy as np

from oracle.gmm import GmmParams, GmmRef
from oracle.pbas import PbasParams, PbasRef
from oracle_runs import OracleRuns, make_job, run, windows
from synth import Scene, preset


def _assemble(H, W, jobs, results, frames):
    masks = np.zeros((frames, H, W), bool)
    state = {}
    for job, res in zip(jobs, results):
        oy, ox, oh, ow = job["own"]
        m = np.unpackbits(res["masks"], axis=1)[:, :oh * ow].reshape(frames, oh, ow)
        masks[:, oy:oy + oh, ox:ox + ow] = m.astype(bool)
        for k, v in res.items():
            if k.startswith("state_"):
                if k not in state:
                    state[k] = np.zeros(v.shape[:-2] + (H, W), v.dtype)
                state[k][..., oy:oy + oh, ox:ox + ow] = v
    return masks, state


def test_windows_partition_the_image():
    for H, W, r, c, m in ((720, 1280, 2, 4, 165), (480, 640, 1, 1, 281), (37, 50, 3, 2, 4), (5, 9, 4, 7, 1)):
        cover = np.zeros((H, W), np.int64)
        for (y0, x0, h, w), (oy, ox, oh, ow) in windows(H, W, r, c, m):
            cover[oy:oy + oh, ox:ox + ow] += 1
            assert y0 <= oy and oy + oh <= y0 + h and x0 <= ox and ox + ow <= x0 + w
            # widened by the margin on every inner side, clipped at the image border
            assert y0 == max(0, oy - m) and x0 == max(0, ox - m)
            assert y0 + h == min(H, oy + oh + m) and x0 + w == min(W, ox + ow + m)
        assert (cover == 1).all()


def test_pbas_windows_reassemble_the_whole_image():
    H, W, N, frames = 26, 34, 4, 12
    p = PbasParams(N=N, T_lower=1.0, T_upper=4.0, seed=21)
    pd = dict(N=N, T_lower=1.0, T_upper=4.0, seed=21)
    ov = dict(H=H, W=W, n_objects=2)
    jobs = [make_job("pbas", "pbas_640x480", ov, pd, frames, H, W, win, own)
            for win, own in windows(H, W, 2, 3, frames - N)]
    results = [run(j) for j in jobs]
    masks, state = _assemble(H, W, jobs, results, frames)
    sc = Scene(preset("pbas_640x480", **ov))
    full = PbasRef(H, W, p)
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        np.testing.assert_array_equal(masks[t], full.step(rgb, D) != 0, err_msg=f"t={t}")
    for k, v in full.state_planes().items():
        if k != "t":
            np.testing.assert_array_equal(state["state_" + k], v, err_msg=k)
    # the margin is needed: windows without it miss writes from outside
    bad = [make_job("pbas", "pbas_640x480", ov, pd, frames, H, W, own, own)
           for _, own in windows(H, W, 2, 3, 0)]
    _, st0 = _assemble(H, W, bad, [run(j) for j in bad], frames)
    assert (st0["state_samples"] != full.state_planes()["samples"]).any()


def test_gmm_bands_in_child_processes(tmp_path):
    H, W, frames = 30, 40, 10
    ov = dict(H=H, W=W)
    pd = dict(Kc=3, Kd=3)
    jobs = [make_job("gmm", "gmm_320x240", ov, pd, frames, H, W, win, own) for win, own in windows(H, W, 3, 1, 0)]
    runs = OracleRuns(jobs, str(tmp_path), procs=3)
    results = [runs.result(i) for i in range(len(jobs))]
    runs.close()
    masks, state = _assemble(H, W, jobs, results, frames)
    sc = Scene(preset("gmm_320x240", **ov))
    full = GmmRef(H, W, GmmParams(Kc=3, Kd=3))
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        np.testing.assert_array_equal(masks[t], full.step(rgb, D) != 0, err_msg=f"t={t}")
    for k, v in full.state_planes().items():
        if k != "t":
            np.testing.assert_array_equal(state["state_" + k], v, err_msg=k)
