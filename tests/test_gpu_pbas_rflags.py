"""PBAS threshold flags: the step kernel carries, in the high nibble of each pixel's fire
byte, which channels' decision threshold R equals its lower bound after the frame, and skips
reading R where all four do.  These runs make R leave its bound and come back (an R_scale at
which the mean minimal distance of noisy pixels crosses R / R_scale), so both the flagged and
the unflagged paths run on every frame, and compare the GPU's R, every other state field and
every mask with the oracle's run from frame 0, bit for bit; the flag path is also taken
across a state read-out (which applies the deferred writes and clears the pending state) and
in the batched streaming launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_pbas_state, log, to_dev  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402
from synth import Scene, preset  # noqa: E402
from test_gpu_parity import _pbas_params_c  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _at_lower(R, p):
    return (R.view(np.uint32) == np.array(p.R_lower, np.float32).view(np.uint32)).all(-1)


@pytest.mark.parametrize("N,H,W,R_scale,frames,readout_at", [
    (8, 45, 131, 30.0, 40, 25),
    (35, 37, 70, 40.0, 60, 50),
    (20, 24, 200, 12.0, 45, -1),
])
def test_r_flags_follow_the_oracle(N, H, W, R_scale, frames, readout_at):
    from paper_2002_00250_amd import fgs
    p = PbasParams(N=N, R_scale=R_scale)
    sc = Scene(preset("pbas_640x480", H=H, W=W))
    m = fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p))
    ref = PbasRef(H, W, p)
    flagged = unflagged = left = returned = 0
    for t in range(frames):
        was = _at_lower(ref.R, p)
        rgb, D, _ = sc.frame(t)
        exp = ref.step(rgb, D)
        m.push(*to_dev(rgb, D))
        assert np.array_equal(m.mask_host(), exp), f"mask differs at frame {t}"
        now = _at_lower(ref.R, p)
        if t > N:
            flagged += int(was.sum())
            unflagged += int((~was).sum())
            left += int((was & ~now).sum())
            returned += int((~was & now).sum())
        if t == readout_at:
            st = m.state()
            res = compare_pbas_state(st, ref.state_planes())
            assert all(v == 0 for v in res.values()), (t, res)
    res = compare_pbas_state(m.state(), ref.state_planes())
    m.close()
    log(f"R flags N={N} {H}x{W} R_scale={R_scale}: pixel-frames with every R at its bound {flagged}, "
        f"others {unflagged}; left the bound {left}, came back {returned}; final state {res}")
    assert all(v == 0 for v in res.values()), res
    assert flagged > 0 and unflagged > 0 and left > 0 and returned > 0


def test_r_flags_in_the_batched_streaming_launch():
    """Eight N = 35 models with their own scenes and R_scale values in one launch of the
    eight-model instance, streaming their state: every model equals its own oracle run."""
    from paper_2002_00250_amd import fgs
    H, W, frames = 29, 97, 50
    stream = torch.cuda.Stream()
    models, refs, scenes = [], [], []
    for i in range(8):
        p = PbasParams(N=35, R_scale=10.0 + 5.0 * i, seed=1000 + i)
        models.append(fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p), stream=stream))
        fgs.fgs_set_cache_policy(models[-1].handle, fgs.FGS_CACHE_STREAM)
        refs.append(PbasRef(H, W, p))
        scenes.append(Scene(preset("pbas_640x480", H=H, W=W, seed=77 + i)))
    outs = torch.empty((8, H, W), dtype=torch.uint8, device="cuda")
    bad = 0
    with torch.cuda.stream(stream):
        for t in range(frames):
            fr = [sc.frame(t) for sc in scenes]
            dev = [to_dev(rgb, D) for rgb, D, _ in fr]
            fgs.push_frames(models, [d[0] for d in dev], [d[1] for d in dev])
            for j, mdl in enumerate(models):
                mdl.mask_into(outs[j])
            got = outs.cpu().numpy()
            for j, (rgb, D, _) in enumerate(fr):
                bad += int((got[j] != refs[j].step(rgb, D)).sum())
    torch.cuda.synchronize()
    res = [compare_pbas_state(mdl.state(), r.state_planes()) for mdl, r in zip(models, refs)]
    for mdl in models:
        mdl.close()
    log(f"R flags, 8 models in one streaming launch, {frames} frames: mask diff {bad}, states {res}")
    assert bad == 0
    assert all(all(v == 0 for v in r.values()) for r in res), res
