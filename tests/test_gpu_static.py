"""GPU static-object detection (reading of Sec. 6's future-work item) against the oracle: the
library's static mask after every push equals oracle.static.StaticRef run on the oracle
model's masks, for GMM and PBAS models on a scene whose objects stop moving, at ragged sizes
(pixel counts not a multiple of 4), through single and batched pushes, with the detector
enabled mid-run, restarted with another M, turned off, and restarted by a state load."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log, to_dev  # noqa: E402
from oracle.gmm import GmmParams, GmmRef  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402
from oracle.static import StaticRef  # noqa: E402
from synth import Scene, preset  # noqa: E402
from test_gpu_parity import _gmm_params_c, _pbas_params_c  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


@pytest.mark.parametrize("kind,H,W,M,enable_at", [
    ("gmm", 48, 80, 6, 0), ("gmm", 37, 53, 1, 5), ("pbas", 41, 67, 9, 0), ("pbas", 30, 35, 3, 12)])
def test_static_mask_equals_oracle(kind, H, W, M, enable_at):
    from paper_2002_00250_amd import fgs
    sc = Scene(preset("gmm_320x240", H=H, W=W, n_objects=2, stop_at=15))
    if kind == "gmm":
        p = GmmParams(Kc=3, Kd=3)
        ref, m = GmmRef(H, W, p), fgs.Model(fgs.FGS_GMM, H, W, _gmm_params_c(p))
    else:
        p = PbasParams(N=6, seed=3)
        ref, m = PbasRef(H, W, p), fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p))
    st = None
    diff = flagged = 0
    for t in range(70):
        if t == enable_at:
            m.static_enable(M)
            st = StaticRef(H, W, M)
        rgb, D, _ = sc.frame(t)
        mask = ref.step(rgb, D)
        m.push(*to_dev(rgb, D))
        if st is not None:
            exp = st.step(mask)
            got = m.static_mask_host()
            diff += int((got != exp).sum())
            flagged += int((exp != 0).sum())
    log(f"static {kind} {H}x{W} M={M} from frame {enable_at}: {diff} pixels differ, {flagged} static pixel-frames")
    assert diff == 0 and flagged > 0
    m.close()


def test_static_batched_restart_off_and_state_load():
    from paper_2002_00250_amd import fgs
    H, W = 29, 45
    sc = Scene(preset("gmm_320x240", H=H, W=W, n_objects=2, stop_at=10))
    stream = torch.cuda.Stream()
    p = GmmParams(Kc=3, Kd=3)
    a = fgs.Model(fgs.FGS_GMM, H, W, _gmm_params_c(p), stream=stream)
    b = fgs.Model(fgs.FGS_GMM, H, W, _gmm_params_c(p), stream=stream)
    ref = GmmRef(H, W, p)
    a.static_enable(4)
    b.static_enable(11)
    sa, sb = StaticRef(H, W, 4), StaticRef(H, W, 11)
    diff = 0
    with torch.cuda.stream(stream):
        for t in range(50):
            rgb, D, _ = sc.frame(t)
            mask = ref.step(rgb, D)
            r, d = to_dev(rgb, D)
            fgs.push_frames([a, b], [r, r], [d, d])
            diff += int((b.static_mask_host() != sb.step(mask)).sum())
            if t == 30:                       # restart a with another M: counting from the next push
                a.static_enable(2)
                sa = StaticRef(H, W, 2)
            else:
                diff += int((a.static_mask_host() != sa.step(mask)).sum())
    assert diff == 0
    # a state load restarts the counters; turning the detector off refuses the mask
    blob = b.state_blob()
    b.set_state(blob)
    with pytest.raises(fgs.FgsError) as e:
        b.static_mask_host()                  # nothing counted since the restart
    assert e.value.status == fgs.FGS_ERR_BAD_STATE
    rgb, D, _ = sc.frame(50)
    mask = ref.step(rgb, D)
    b.push(*to_dev(rgb, D))
    np.testing.assert_array_equal(b.static_mask_host(), StaticRef(H, W, 11).step(mask))
    b.static_enable(0)
    with pytest.raises(fgs.FgsError) as e:
        b.static_mask_host()
    assert e.value.status == fgs.FGS_ERR_BAD_STATE
    for bad in (-1, 65536):
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_static_enable(b.handle, bad)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    a.close()
    b.close()
