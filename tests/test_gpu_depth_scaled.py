"""Depth at another resolution than RGB (Sec. 4.3: upscaled to the RGB grid): the kernels'
in-register nearest-neighbour upscale against the oracle fed the explicitly upscaled map,
with the paper's own GMM settings (7 colour / 3 depth Gaussians, learning rate 0.001) and
PBAS N = 20."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_gmm_state, compare_pbas_state, log  # noqa: E402
from oracle.depth import upscale_nearest  # noqa: E402
from oracle.gmm import GmmParams, GmmRef  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402
from synth import Scene, preset  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _low_depth(D, Hd, Wd):
    """Sensor-side depth at Hd x Wd: decimate the scene's full-resolution depth."""
    H, W = D.shape
    ys = (np.arange(Hd) * H) // Hd
    xs = (np.arange(Wd) * W) // Wd
    return np.ascontiguousarray(D[ys][:, xs])


@pytest.mark.parametrize("H,W,Hd,Wd,mode", [(72, 128, 48, 85, "device"), (48, 64, 24, 32, "host"),
                                            (45, 80, 30, 53, "device"), (40, 40, 40, 40, "device")])
def test_gmm_paper_settings_with_scaled_depth(H, W, Hd, Wd, mode):
    from paper_2002_00250_amd import fgs
    p = GmmParams(Kc=7, Kd=3, alpha=0.001)
    c = fgs.fgs_gmm_params_default()
    c.Kc, c.Kd, c.alpha = 7, 3, 0.001
    sc = Scene(preset("hd_1280x720", H=H, W=W))
    ref = GmmRef(H, W, p)
    m = fgs.Model(fgs.FGS_GMM, H, W, c)
    diff = 0
    for t in range(30):
        rgb, D, _ = sc.frame(t)
        Dl = _low_depth(D, Hd, Wd)
        exp = ref.step(rgb, upscale_nearest(Dl, H, W))
        if mode == "host":
            m.push(rgb, Dl)
        else:
            m.push(torch.from_numpy(rgb).cuda(), torch.from_numpy(Dl.view(np.int16)).cuda())
        diff += int((m.mask_host() != exp).sum())
    n, bad, neq = compare_gmm_state(m.state(), ref.state_planes())
    log(f"gmm 7/3 alpha 0.001 rgb {H}x{W} depth {Hd}x{Wd} {mode}: mask diff {diff}, state bad {bad}, not bit-equal {neq}")
    assert diff == 0 and bad == 0
    m.close()


@pytest.mark.parametrize("H,W,Hd,Wd", [(72, 128, 48, 85), (37, 70, 25, 47)])
def test_pbas_with_scaled_depth(H, W, Hd, Wd):
    from paper_2002_00250_amd import fgs
    p = PbasParams(N=20, seed=99)
    c = fgs.fgs_pbas_params_default()
    c.N, c.seed = 20, 99
    sc = Scene(preset("pbas_640x480", H=H, W=W))
    ref = PbasRef(H, W, p)
    m = fgs.Model(fgs.FGS_PBAS, H, W, c)
    diff = 0
    for t in range(45):
        rgb, D, _ = sc.frame(t)
        Dl = _low_depth(D, Hd, Wd)
        exp = ref.step(rgb, upscale_nearest(Dl, H, W))
        m.push(torch.from_numpy(rgb).cuda(), torch.from_numpy(Dl.view(np.int16)).cuda())
        diff += int((m.mask_host() != exp).sum())
    res = compare_pbas_state(m.state(), ref.state_planes())
    log(f"pbas N=20 rgb {H}x{W} depth {Hd}x{Wd}: mask diff {diff}, state {res}")
    assert diff == 0 and all(v == 0 for k, v in res.items() if not k.endswith("bits"))
    m.close()


def test_scaled_depth_rejects_bad_sizes():
    from paper_2002_00250_amd import fgs
    m = fgs.Model(fgs.FGS_GMM, 8, 8)
    r = np.zeros((8, 8, 3), np.uint8)
    d = np.zeros((16, 16), np.uint16)
    with pytest.raises(fgs.FgsError) as e:      # host depth larger than the frame
        m.push(r, d)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    m.close()
