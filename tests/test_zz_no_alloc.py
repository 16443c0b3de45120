"""fgs_copy_state_noalloc (the allocation-free state copy) against fgs_copy_state.

Each case pushes frames into a model, then takes its serialised state both ways through
the C ABI and requires the two blobs to be identical byte for byte: a host destination
(staged through the library's fixed device buffer), then a device destination.  Two
calls in a row on one GPU, the second with a smaller model, so the second call reads a
buffer that still holds the first call's larger payload.  A payload beyond the buffer is
refused with UNSUPPORTED and leaves the destination untouched, while a device
destination of the same model has no limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log, to_dev  # noqa: E402
from synth import Scene, preset  # noqa: E402


def _model(fgs, algo, H, W, frames, **kw):
    if algo == "gmm":
        p = fgs.fgs_gmm_params_default()
        for k, v in kw.items():
            setattr(p, k, v)
        m = fgs.Model(fgs.FGS_GMM, H, W, p)
    else:
        p = fgs.fgs_pbas_params_default()
        for k, v in kw.items():
            setattr(p, k, v)
        m = fgs.Model(fgs.FGS_PBAS, H, W, p)
    sc = Scene(preset("pbas_640x480", H=H, W=W))
    for t in range(frames):
        rgb, D, _ = sc.frame(t)
        m.push(*to_dev(rgb, D))
    return m


def _both_ways(fgs, m):
    n = fgs.fgs_state_size(m.handle)
    ref = np.empty(n, np.uint8)
    fgs.fgs_copy_state(m.handle, ref.ctypes.data, n, fgs.FGS_MEM_HOST)
    got = np.full(n, 0xA5, np.uint8)
    fgs.fgs_copy_state_noalloc(m.handle, got.ctypes.data, n, fgs.FGS_MEM_HOST)
    dev = torch.full((n,), 0x5A, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    fgs.fgs_copy_state_noalloc(m.handle, dev.data_ptr(), n, fgs.FGS_MEM_DEVICE)
    m.sync()
    return ref, got, dev.cpu().numpy()


@pytest.mark.parametrize("algo,big,small,kw", [
    ("pbas", (120, 200), (37, 70), dict(N=20)),
    ("pbas", (96, 160), (29, 51), dict(N=12, gradient=1)),   # the gradient variant's export
    ("gmm", (150, 256), (33, 45), dict(Kc=5, Kd=5)),
    ("gmm", (64, 100), (20, 30), dict(Kc=7, Kd=3, var_mode=1)),
])
def test_noalloc_copy_equals_copy_twice_shrinking(algo, big, small, kw):
    from paper_2002_00250_amd import fgs
    fgs.lib()
    frames = 30
    for H, W in (big, small):
        m = _model(fgs, algo, H, W, frames, **kw)
        ref, got, dev = _both_ways(fgs, m)
        nh = int((got != ref).sum())
        nd = int((dev != ref).sum())
        log(f"noalloc {algo} {H}x{W}: {ref.size} bytes, host copy differs in {nh}, device copy in {nd}")
        assert nh == 0 and nd == 0
        # the model keeps running after an allocation-free copy (a PBAS copy applies the
        # deferred neighbour writes, as fgs_copy_state does)
        sc = Scene(preset("pbas_640x480", H=H, W=W))
        rgb, D, _ = sc.frame(frames)
        m.push(*to_dev(rgb, D))
        ref2, got2, _ = _both_ways(fgs, m)
        assert np.array_equal(ref2, got2)
        m.close()


def test_noalloc_copy_refuses_payload_beyond_buffer():
    from paper_2002_00250_amd import fgs
    fgs.lib()
    # GMM Kc = Kd = 5 at 640x512: 160 B of state per pixel, 52 MB; at 720x640: 74 MB > 64 MiB
    m = _model(fgs, "gmm", 720, 640, 2, Kc=5, Kd=5)
    n = fgs.fgs_state_size(m.handle)
    assert n - 64 > fgs.FGS_NOALLOC_STAGING_BYTES
    dst = np.full(n, 0x33, np.uint8)
    with pytest.raises(fgs.FgsError) as ei:
        fgs.fgs_copy_state_noalloc(m.handle, dst.ctypes.data, n, fgs.FGS_MEM_HOST)
    assert ei.value.status == fgs.FGS_ERR_UNSUPPORTED
    assert (dst == 0x33).all()
    ref = np.empty(n, np.uint8)
    fgs.fgs_copy_state(m.handle, ref.ctypes.data, n, fgs.FGS_MEM_HOST)
    dev = torch.empty((n,), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    fgs.fgs_copy_state_noalloc(m.handle, dev.data_ptr(), n, fgs.FGS_MEM_DEVICE)
    m.sync()
    assert np.array_equal(dev.cpu().numpy(), ref)
    # a wrong size is refused as by fgs_copy_state
    with pytest.raises(fgs.FgsError) as ei:
        fgs.fgs_copy_state_noalloc(m.handle, dst.ctypes.data, n - 1, fgs.FGS_MEM_HOST)
    assert ei.value.status == fgs.FGS_ERR_INVALID_ARG
    m.close()
