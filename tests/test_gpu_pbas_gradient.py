"""GPU parity of the PBAS gradient-magnitude variant (opt-in: the base method's second
feature on the colour channels, reading R-23) against the oracle: every mask and the final
state (sample values and magnitudes exact, float D, S, R, T within 1e-4 relative, expected
bit-equal) at ragged sizes and several N, host and device frames; a state round trip in
the middle of a run; in-place state fields; a batched call mixing it with plain models;
alpha = 0 equal to the plain variant."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_pbas_grad_state, compare_pbas_state, log, to_dev  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402
from synth import Scene, preset  # noqa: E402
from test_gpu_parity import MASK_TOL, _pbas_params_c  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _all_zero(res):
    return all(v == 0 for v in res.values())


@pytest.mark.parametrize("H,W,N,frames,mode", [
    (37, 71, 6, 40, "device"),
    (21, 70, 20, 50, "device"),
    (9, 130, 35, 60, "host"),
    (70, 90, 12, 45, "device"),
    (1, 1, 2, 12, "device"),
    (5, 3, 64, 75, "device"),
])
def test_gradient_parity_trajectories(H, W, N, frames, mode):
    from paper_2002_00250_amd import fgs
    p = PbasParams(N=N, gradient=True, seed=0x51 + N)
    sc = Scene(preset("pbas_640x480", H=H, W=W))
    ref = PbasRef(H, W, p)
    m = fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p))
    diff = 0
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        exp = ref.step(rgb, D)
        if mode == "host":
            m.push(rgb, D)
        else:
            m.push(*to_dev(rgb, D))
        diff += int((m.mask_host() != exp).sum())
    res = compare_pbas_grad_state(m.state(), ref.state_planes())
    m.close()
    log(f"pbas gradient {H}x{W} N={N} {frames} frames ({mode}): mask diff {diff}/{frames * H * W}, state {res}")
    assert diff <= MASK_TOL * frames * H * W and _all_zero(res)


def test_gradient_state_round_trip_and_fields():
    from paper_2002_00250_amd import fgs
    H, W = 33, 67
    p = PbasParams(N=8, gradient=True, grad_alpha=7.0, seed=77)
    sc = Scene(preset("pbas_640x480", H=H, W=W))
    frames = [sc.frame(t)[:2] for t in range(36)]
    a = fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p))
    for rgb, D in frames[:20]:
        a.push(*to_dev(rgb, D))
    blob = a.state_blob()                       # applies the pending neighbour writes
    st = fgs.unpack_state(blob)
    assert st["gradient"] and st["gsum"].shape == (3,)
    b = fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p))
    b.set_state(blob)
    np.testing.assert_array_equal(b.state_blob(), blob)
    ref = PbasRef(H, W, p)
    for rgb, D in frames:
        ref.step(rgb, D)
    for rgb, D in frames[20:]:
        for mdl in (a, b):
            mdl.push(*to_dev(rgb, D))
        np.testing.assert_array_equal(a.mask_host(), b.mask_host())
    np.testing.assert_array_equal(a.state_blob(), b.state_blob())
    res = compare_pbas_grad_state(b.state(), ref.state_planes())
    log(f"pbas gradient round trip: state {res}")
    assert _all_zero(res)
    a.close()
    b.close()


def test_gradient_in_place_fields_equal_the_serialised_state():
    # fields taken with neighbour writes still deferred: the call applies them first
    from paper_2002_00250_amd import fgs
    from test_gpu_state_fields import _values
    H, W = 17, 40
    p = PbasParams(N=5, gradient=True, seed=5)
    sc = Scene(preset("pbas_640x480", H=H, W=W))
    m = fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p))
    for t in range(12):
        m.push(*to_dev(*sc.frame(t)[:2]))
    fields = fgs.fgs_get_state(m.handle)
    fgs.fgs_sync(m.handle)
    st = m.state()
    names = set()
    for f in fields:
        name, k, j = f["name"], f["index"], f["sub"]
        exp = st[name][k, j] if name == "dhist" else st[name][k]
        np.testing.assert_array_equal(_values(f, H, W), exp, err_msg=f"{name}[{k}][{j}]")
        names.add(name)
    assert names == {"samples", "gsamples", "dhist", "R", "T", "S"} and len(fields) == 6 * p.N + 12
    m.close()


def test_gradient_model_in_a_batched_call_and_alpha_zero():
    # push_frames with a gradient model among plain PBAS models: each equals its oracle;
    # the gradient model at alpha = 0 equals the plain model on the same frames
    from paper_2002_00250_amd import fgs
    H, W = 29, 75
    stream = torch.cuda.Stream()
    specs = [PbasParams(N=10, seed=9), PbasParams(N=10, seed=9, gradient=True, grad_alpha=0.0),
             PbasParams(N=10, seed=10, gradient=True), PbasParams(N=12, seed=11)]
    models = [fgs.Model(fgs.FGS_PBAS, H, W, _pbas_params_c(p), stream=stream) for p in specs]
    refs = [PbasRef(H, W, p) for p in specs]
    sc = Scene(preset("pbas_640x480", H=H, W=W, seed=33))
    diffs = [0] * len(specs)
    same = 0
    with torch.cuda.stream(stream):
        for t in range(30):
            rgb, D, _ = sc.frame(t)
            r, d = to_dev(rgb, D)
            fgs.push_frames(models, [r] * 4, [d] * 4)
            masks = [m.mask_host() for m in models]
            for i, (ref, mk) in enumerate(zip(refs, masks)):
                diffs[i] += int((mk != ref.step(rgb, D)).sum())
            same += int((masks[0] != masks[1]).sum())
    res = [compare_pbas_state(models[i].state(), refs[i].state_planes()) if not specs[i].gradient
           else compare_pbas_grad_state(models[i].state(), refs[i].state_planes()) for i in range(4)]
    log(f"gradient in a batched call: mask diffs {diffs}, alpha 0 vs plain {same}, state {res}")
    assert diffs == [0, 0, 0, 0] and same == 0 and all(_all_zero(r) for r in res)
    for m in models:
        m.close()
