"""Segmentation quality on the synthetic stand-ins for the paper's evaluation categories
(Sec. 5: colour camouflage, shadows, illumination changes), GMM and PBAS, with and without
depth, through the GPU path; indicators PWC / FNR / FPR / Si as defined in Sec. 5.

The paper's data is not available, so the numbers are not comparable to Tables 2-3; the
test checks the qualitative claim that depth matters most for colour camouflage: an object
whose colour equals the background is found only when depth takes part."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log  # noqa: E402
from oracle.metrics import confusion, indicators  # noqa: E402
from synth import Scene, preset  # noqa: E402

SCENES = {
    "colour camouflage": dict(n_objects=0, camouflage=True, illumination=False),
    "shadows": dict(n_objects=4, shadows=True),
    "illumination": dict(n_objects=3, illumination=True),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _evaluate(algo, params, cfg, use_depth, frames=160, skip=60):
    from paper_2002_00250_amd import fgs
    sc = Scene(cfg)
    m = fgs.Model(algo, cfg.H, cfg.W, params)
    conf = np.zeros(4, np.int64)
    for t in range(frames):
        rgb, D, gt = sc.frame(t)
        if not use_depth:
            D = np.zeros_like(D)
        m.push(torch.from_numpy(rgb).cuda(), torch.from_numpy(D.view(np.int16)).cuda())
        if t >= skip:
            conf += confusion(m.mask_host(), gt)
    m.close()
    return indicators(*conf)


def test_quality_table_and_camouflage_claim():
    from paper_2002_00250_amd import fgs
    gp = fgs.fgs_gmm_params_default()
    pp = fgs.fgs_pbas_params_default()
    rows = {}
    for name, kw in SCENES.items():
        cfg = preset("gmm_320x240", **kw)
        for algo, prm, tag in ((fgs.FGS_GMM, gp, "GMM"), (fgs.FGS_PBAS, pp, "PBAS")):
            for use_depth in (False, True):
                r = _evaluate(algo, prm, cfg, use_depth)
                rows[(name, tag + (" + RGBD" if use_depth else ""))] = r
    log("| sequence | method | PWC | FNR | FPR | Si |")
    for (seq, meth), r in rows.items():
        log(f"| {seq} | {meth} | {r['PWC']:.2f} | {r['FNR']:.4f} | {r['FPR']:.4f} | {r['Si']:.2f} |")
    for tag in ("GMM", "PBAS"):
        rgb = rows[("colour camouflage", tag)]
        rgbd = rows[("colour camouflage", tag + " + RGBD")]
        assert rgb["FNR"] > 0.9           # colour alone cannot see the object
        assert rgbd["FNR"] < 0.5          # depth finds it
        assert rgbd["Si"] > rgb["Si"] + 0.4
