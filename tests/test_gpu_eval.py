"""Evaluation counters (fgs_eval_accumulate / fgs_eval_read): the device-accumulated
confusion counts equal the oracle's (Sec. 5 definitions) exactly, for host and strided
device ground truth, ragged sizes, per-frame resets, and the full 1280x720 frame."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log  # noqa: E402
from oracle.metrics import confusion, indicators  # noqa: E402
from synth import Scene, preset  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _model(algo, H, W):
    from paper_2002_00250_amd import fgs
    if algo == "gmm":
        p = fgs.fgs_gmm_params_default()
        return fgs.Model(fgs.FGS_GMM, H, W, p)
    p = fgs.fgs_pbas_params_default()
    p.N = 6
    return fgs.Model(fgs.FGS_PBAS, H, W, p)


@pytest.mark.parametrize("algo", ["gmm", "pbas"])
def test_counts_equal_oracle_ragged(algo):
    H, W = 61, 97
    sc = Scene(preset("gmm_320x240", H=H, W=W, seed=11))
    m = _model(algo, H, W)
    total = np.zeros(4, np.int64)
    for t in range(14):
        rgb, dep, gt = sc.frame(t)
        m.push(rgb, dep)
        m.eval_accumulate(gt)                      # host ground truth
        ref = confusion(m.mask_host(), gt)
        total += ref
        if t % 5 == 4:                              # per-frame read with reset
            got = m.eval_read(reset=True)
            assert got == tuple(int(v) for v in total), (t, got, total)
            total[:] = 0
    assert m.eval_read() == tuple(int(v) for v in total)
    assert sum(m.eval_read()) == (14 % 5) * H * W
    m.close()


def test_strided_device_ground_truth_and_errors():
    from paper_2002_00250_amd import fgs
    H, W = 40, 70
    sc = Scene(preset("gmm_320x240", H=H, W=W, seed=5))
    m = _model("gmm", H, W)
    with pytest.raises(fgs.FgsError) as e:                 # no mask before the first push
        m.eval_accumulate(np.zeros((H, W), np.uint8))
    assert e.value.status == fgs.FGS_ERR_BAD_STATE
    assert m.eval_read() == (0, 0, 0, 0)
    wide = torch.zeros((H, W + 13), dtype=torch.uint8, device="cuda")
    total = np.zeros(4, np.int64)
    for t in range(9):
        rgb, dep, gt = sc.frame(t)
        m.push(rgb, dep)
        wide[:, :W] = torch.from_numpy(gt).cuda()
        wide[:, W:] = 255                                  # outside the view: must not count
        m.eval_accumulate(wide[:, :W])
        total += confusion(m.mask_host(), gt)
    assert m.eval_read() == tuple(int(v) for v in total)
    with pytest.raises(fgs.FgsError) as e:
        fgs.fgs_eval_accumulate(m.handle, wide.data_ptr(), W - 1, fgs.FGS_MEM_DEVICE)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    m.close()


def test_full_frame_matches_oracle_masks():
    # 1280x720, GMM K=5: the counts of the GPU masks equal the counts of the oracle's
    # own masks on the same frames (the masks themselves are bit-exact).
    from oracle.gmm import GmmParams, GmmRef
    from paper_2002_00250_amd import fgs
    sc = Scene(preset("hd_1280x720"))
    H, W = sc.cfg.H, sc.cfg.W
    p = fgs.fgs_gmm_params_default()
    p.Kc = p.Kd = 5
    m = fgs.Model(fgs.FGS_GMM, H, W, p)
    ref = GmmRef(H, W, GmmParams(Kc=5, Kd=5))
    total = np.zeros(4, np.int64)
    for t in range(4):
        rgb, dep, gt = sc.frame(t)
        m.push(rgb, dep)
        m.eval_accumulate(gt)
        total += confusion(ref.step(rgb, dep), gt)
    got = m.eval_read()
    log(f"720p GMM K=5, 4 frames: counts {got}, indicators "
        f"{ {k: round(v, 4) for k, v in indicators(*got).items()} }")
    assert got == tuple(int(v) for v in total)
    m.close()
