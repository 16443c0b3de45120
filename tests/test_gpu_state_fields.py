"""fgs_get_state: the in-place fields of the model's device state read back through their
addresses and strides equal the serialised state (fgs_copy_state) bit for bit, for GMM
(both variance layouts, the paper's 7/3) and PBAS (N not a multiple of 4, with neighbour
writes still deferred when the fields are taken)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from synth import Scene, preset  # noqa: E402

_HIP = None


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield


def _read_device(ptr: int, nbytes: int) -> np.ndarray:
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(nbytes, np.uint8)
    assert _HIP.hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0   # device to host
    return out


def _values(f, H, W):
    npix = H * W
    e, s = f["elem_bytes"], f["pixel_stride"]
    raw = _read_device(f["base"], (npix - 1) * s + e)
    elems = np.lib.stride_tricks.as_strided(raw, shape=(npix, e), strides=(s, 1)).copy()
    dt = {1: np.float32, 2: np.uint32, 3: np.uint16}[f["dtype"]]
    return elems.view(dt).reshape(H, W)


def _canonical(st, f):
    name, k, c = f["name"], f["index"], f["sub"]
    a = np.asarray(st[name])
    if name == "mu_c" or (name == "v_c" and a.ndim == 4):
        return a[k, c]
    return a[k]


def _check_all(m, H, W):
    from paper_2002_00250_amd import fgs
    fields = fgs.fgs_get_state(m.handle)
    fgs.fgs_sync(m.handle)
    st = m.state()
    seen = set()
    for f in fields:
        got, exp = _values(f, H, W), _canonical(st, f)
        assert got.shape == exp.shape
        np.testing.assert_array_equal(got.view(np.uint8), np.ascontiguousarray(exp).view(np.uint8),
                                      err_msg=f"{f['name']}[{f['index']}][{f['sub']}]")
        seen.add((f["name"], f["index"], f["sub"]))
    return fields, seen


@pytest.mark.parametrize("Kc,Kd,var_mode", [(5, 5, 0), (7, 3, 0), (3, 3, 1)])
def test_gmm_fields_equal_serialised_state(Kc, Kd, var_mode):
    from paper_2002_00250_amd import fgs
    H, W = 37, 83
    p = fgs.fgs_gmm_params_default()
    p.Kc, p.Kd, p.var_mode = Kc, Kd, var_mode
    m = fgs.Model(fgs.FGS_GMM, H, W, p)
    sc = Scene(preset("gmm_320x240", H=H, W=W, n_objects=2))
    for t in range(15):
        m.push(*sc.frame(t)[:2])
    fields, seen = _check_all(m, H, W)
    nv = 3 if var_mode else 1
    assert len(fields) == Kc * (4 + nv) + 3 * Kd == len(seen)
    m.close()


def test_pbas_fields_equal_serialised_state_with_deferred_writes():
    from paper_2002_00250_amd import fgs
    H, W = 29, 70
    p = fgs.fgs_pbas_params_default()
    p.N = 35
    m = fgs.Model(fgs.FGS_PBAS, H, W, p)
    sc = Scene(preset("pbas_640x480", H=H, W=W, n_objects=2))
    for t in range(42):
        m.push(*sc.frame(t)[:2])
    n = ctypes.c_int32()
    small = (fgs.fgs_state_field * 3)()
    with pytest.raises(fgs.FgsError) as e:
        fgs._check(fgs._load().fgs_get_state(ctypes.c_void_p(m.handle), small, 3, ctypes.byref(n)))
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG and n.value == 2 * 35 + 12
    fields, seen = _check_all(m, H, W)   # applies frame 41's deferred neighbour writes first
    assert len(fields) == 2 * 35 + 12 == len(seen)
    # one more frame, then the same addresses hold the new state
    m.push(*sc.frame(42)[:2])
    _check_all(m, H, W)
    m.close()
