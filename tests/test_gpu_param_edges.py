"""GPU parity at the edges of the accepted parameter ranges: the kernels and the oracle
must agree bit for bit when rates, thresholds and bounds sit at extreme values (fast and
slow rates, tiny and huge thresholds, a background set of one or of all Gaussians, no depth
weight, other depth full scales; PBAS with every sample required or one, fixed rates,
thresholds below one code level or above the byte range)."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log  # noqa: E402
from oracle.gmm import GmmParams  # noqa: E402
from oracle.pbas import PbasParams  # noqa: E402
from synth import preset  # noqa: E402
from test_gpu_parity import _run_gmm_pair, _run_pbas_pair  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


GMM_EDGES = {
    "fast rate": GmmParams(Kc=3, Kd=3, alpha=0.9),
    "slow rate": GmmParams(Kc=5, Kd=5, alpha=1e-6),
    "background = first Gaussian": GmmParams(Kc=5, Kd=5, T_bg=0.01),
    "background = nearly all": GmmParams(Kc=5, Kd=5, T_bg=0.999),
    "huge lambda": GmmParams(Kc=3, Kd=3, lam=60.0),
    "tiny lambda": GmmParams(Kc=3, Kd=3, lam=0.05),
    "new Gaussian weight 1, no floor gap": GmmParams(Kc=4, Kd=4, w_init=1.0, v_init_c=12.0, v_init_d=1.0),
    "no depth weight": GmmParams(Kc=3, Kd=3, w_depth=0.0),
    "depth code = D >> 8 scale": GmmParams(Kc=3, Kd=3, depth_max_mm=65535),
    "short depth range": GmmParams(Kc=3, Kd=3, depth_max_mm=700),
    "density threshold 0": GmmParams(Kc=3, Kd=3, decision=1, density_threshold=0.0),
    "per-channel, fast rate": GmmParams(Kc=3, Kd=3, alpha=0.5, var_mode=1),
}

PBAS_EDGES = {
    "every sample must match": PbasParams(N=6, min_matches=6),
    "one match suffices": PbasParams(N=6, min_matches=1),
    "fixed rate": PbasParams(N=8, T_lower=5.0, T_upper=5.0),
    "update every frame": PbasParams(N=8, T_lower=1.0, T_upper=1.0),
    "no R adaptation": PbasParams(N=8, R_incdec=0.0),
    "tiny T increments": PbasParams(N=8, T_inc=1e-6, T_dec=1e-6),
    "threshold below one level": PbasParams(N=8, R_lower=(0.5, 0.5, 0.5, 0.5)),
    "threshold above the byte range": PbasParams(N=8, R_lower=(300.0, 300.0, 300.0, 300.0)),
    "short depth range, N 35": PbasParams(N=35, depth_max_mm=700),
}


@pytest.mark.parametrize("name", list(GMM_EDGES))
def test_gmm_edges(name):
    cfg = preset("gmm_320x240", H=37, W=83, n_objects=3, illumination=True, camouflage=True)
    p = GMM_EDGES[name]
    diff, total, n, bad, neq = _run_gmm_pair(cfg, p, 30)
    log(f"gmm edge '{name}': mask diff {diff}/{total}, state bad {bad}/{n}, not bit-equal {neq}")
    if p.decision == 1:
        assert diff <= 1e-4 * total and bad == 0 and neq == 0
    else:
        assert diff == 0 and bad == 0 and neq == 0


@pytest.mark.parametrize("name", list(PBAS_EDGES))
def test_pbas_edges(name):
    p = PBAS_EDGES[name]
    cfg = preset("pbas_640x480", H=37, W=83, n_objects=3)
    diff, total, res = _run_pbas_pair(cfg, p, p.N + 25)
    log(f"pbas edge '{name}': mask diff {diff}/{total}, state {res}")
    assert diff == 0 and all(v == 0 for v in res.values()), res
