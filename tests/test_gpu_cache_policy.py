"""fgs_set_cache_policy: the kernels' cached and non-temporal (streaming) instances give
identical masks and state, and both equal the oracle, for GMM (the default instance, the
run-time-options instance, per-channel variances) and PBAS (two register classes)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_gmm_state, compare_pbas_state, log, to_dev  # noqa: E402
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


def _gmm_c(p):
    from paper_2002_00250_amd import fgs
    c = fgs.fgs_gmm_params_default()
    c.Kc, c.Kd, c.rho_mode, c.decision, c.var_mode = p.Kc, p.Kd, p.rho_mode, p.decision, p.var_mode
    return c


def _pbas_c(p):
    from paper_2002_00250_amd import fgs
    c = fgs.fgs_pbas_params_default()
    c.N = p.N
    return c


CASES = [("gmm", GmmParams(Kc=5, Kd=5)), ("gmm", GmmParams(Kc=7, Kd=3, rho_mode=1)),
         ("gmm", GmmParams(Kc=3, Kd=3, var_mode=1)), ("pbas", PbasParams(N=20)), ("pbas", PbasParams(N=35))]


@pytest.mark.parametrize("kind,p", CASES, ids=[f"{k}-{i}" for i, (k, _) in enumerate(CASES)])
def test_keep_and_stream_identical_and_equal_the_oracle(kind, p):
    from paper_2002_00250_amd import fgs
    H, W = 45, 131
    sc = Scene(preset("pbas_640x480", H=H, W=W, n_objects=3))
    algo = fgs.FGS_GMM if kind == "gmm" else fgs.FGS_PBAS
    c = _gmm_c(p) if kind == "gmm" else _pbas_c(p)
    keep, stream = fgs.Model(algo, H, W, c), fgs.Model(algo, H, W, c)
    fgs.fgs_set_cache_policy(keep.handle, fgs.FGS_CACHE_KEEP)
    fgs.fgs_set_cache_policy(stream.handle, fgs.FGS_CACHE_STREAM)
    ref = GmmRef(H, W, p) if kind == "gmm" else PbasRef(H, W, p)
    frames = 30 if kind == "gmm" else p.N + 12
    diff = 0
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        exp = ref.step(rgb, D)
        for m in (keep, stream):
            m.push(*to_dev(rgb, D))
        a, b = keep.mask_host(), stream.mask_host()
        np.testing.assert_array_equal(a, b, err_msg=f"t={t}")
        diff += int((a != exp).sum())
    np.testing.assert_array_equal(keep.state_blob(), stream.state_blob())
    if kind == "gmm":
        n, bad, neq = compare_gmm_state(keep.state(), ref.state_planes())
        ok = bad == 0 and neq == 0
    else:
        res = compare_pbas_state(keep.state(), ref.state_planes())
        ok = all(v == 0 for v in res.values())
    log(f"cache policy {kind} {p}: keep == stream, mask diff vs oracle {diff}")
    assert diff == 0 and ok
    with pytest.raises(fgs.FgsError) as e:
        fgs.fgs_set_cache_policy(keep.handle, 3)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    keep.close()
    stream.close()
