"""The C ABI library loads and exports every entry point include/fgs.h declares, and the
binding's structures match the header's layout (no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fgs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fgs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libfgs():
    from paper_2002_00250_amd import build, fgs
    if not os.path.exists(fgs.LIB_PATH):
        build.build(verbose=False)
    return ctypes.CDLL(fgs.LIB_PATH)


def test_every_declared_symbol_is_exported(libfgs):
    names = declared_functions()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(libfgs, n)]
    assert not missing, missing


def test_binding_covers_header_and_struct_sizes(libfgs):
    from paper_2002_00250_amd import fgs
    for n in declared_functions():
        assert hasattr(fgs, n), n
    assert ctypes.sizeof(fgs.fgs_gmm_params) == 72
    assert ctypes.sizeof(fgs.fgs_pbas_params) == 80
    p = fgs.fgs_gmm_params_default()
    assert p.struct_size == 72 and (p.Kc, p.Kd) == (3, 3) and (p.rho_mode, p.decision, p.var_mode) == (0, 0, 0)
    q = fgs.fgs_pbas_params_default()
    assert q.struct_size == 80 and q.N == 20 and list(q.R_lower) == [18, 18, 18, 4]


def test_defaults_match_oracle_readings(libfgs):
    from oracle.gmm import GmmParams
    from oracle.pbas import PbasParams
    from paper_2002_00250_amd import fgs
    import numpy as np
    g, og = fgs.fgs_gmm_params_default(), GmmParams()
    for a, b in (("alpha", "alpha"), ("lambda_", "lam"), ("T_bg", "T_bg"), ("w_init", "w_init"),
                 ("v_init_c", "v_init_c"), ("v_min_c", "v_min_c"), ("v_init_d", "v_init_d"),
                 ("v_min_d", "v_min_d"), ("w_depth", "w_depth"), ("depth_max_mm", "depth_max_mm"),
                 ("rho_mode", "rho_mode"), ("decision", "decision"), ("density_scale", "density_scale"),
                 ("density_threshold", "density_threshold"), ("var_mode", "var_mode")):
        assert np.float32(getattr(g, a)) == np.float32(getattr(og, b)), a
    q, oq = fgs.fgs_pbas_params_default(), PbasParams()
    for a in ("N", "min_matches", "R_incdec", "R_scale", "T_inc", "T_dec", "T_lower", "T_upper",
              "depth_max_mm", "seed", "gradient", "grad_alpha"):
        assert np.float64(getattr(q, a)) == np.float64(np.float32(getattr(oq, a))) or \
            getattr(q, a) == getattr(oq, a), a


def test_errors_without_device(libfgs):
    from paper_2002_00250_amd import fgs
    # the median filter checks its arguments before touching a device; an empty image is a no-op
    for args in [(16, 0, 16, 0, 4, 4, 8), (16, 4, 16, 4, 4, 4, -1), (16, 3, 32, 4, 4, 4, 1),
                 (16, 4, 32, 4, -1, 4, 1), (0, 4, 32, 4, 4, 4, 1), (16, 4, 18, 4, 4, 4, 1),
                 (16, 1 << 30, 1 << 40, 1 << 30, 1 << 30, 1 << 30, 1)]:
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_mask_median(*args)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG, args
    fgs.fgs_mask_median(0, 0, 0, 0, 0, 7, 3)
    fgs.fgs_mask_median(0, 0, 0, 0, 7, 0, 3)
    # batched pushes: an empty batch and a NULL model are refused before any device work
    for models in ([], [0], [0, 0]):
        n = len(models)
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_push_frames(models, [16] * n, [96] * n, [16] * n, [64] * n)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG, models
    with pytest.raises(fgs.FgsError) as e:
        fgs.fgs_create(fgs.FGS_GMM, 0, 10)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    p = fgs.fgs_pbas_params_default()
    p.N = 65
    with pytest.raises(fgs.FgsError) as e:
        fgs.fgs_create(fgs.FGS_PBAS, 10, 10, p)
    assert "N = 65" in str(e.value)
    # a zero T increment would turn T_inc / d_bar into 0/0 where d_bar = 0: refused
    for field, bad in (("T_inc", 0.0), ("T_dec", 0.0), ("T_lower", 0.0), ("min_matches", 0),
                       ("R_incdec", 1.0)):
        p = fgs.fgs_pbas_params_default()
        setattr(p, field, bad)
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_create(fgs.FGS_PBAS, 10, 10, p)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG, field
    assert fgs.fgs_status_str(4) == "bad state"
    # a struct_size that is neither the current nor the earlier (52-byte) layout
    g = fgs.fgs_gmm_params_default()
    g.struct_size = 53
    with pytest.raises(fgs.FgsError) as e:
        fgs.fgs_create(fgs.FGS_GMM, 8, 8, g)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG and "struct_size 53" in str(e.value)
    g = fgs.fgs_gmm_params_default()
    g.rho_mode = 3
    with pytest.raises(fgs.FgsError) as e:
        fgs.fgs_create(fgs.FGS_GMM, 8, 8, g)
    assert e.value.status == fgs.FGS_ERR_INVALID_ARG
    for field, bad in (("decision", 2), ("density_scale", 0.0), ("density_threshold", -1.0), ("var_mode", 2)):
        g = fgs.fgs_gmm_params_default()
        setattr(g, field, bad)
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_create(fgs.FGS_GMM, 8, 8, g)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG, field
    # the adjoint is derived for rho = alpha and the Z score
    for field in ("rho_mode", "decision", "var_mode"):
        g = fgs.fgs_gmm_params_default()
        setattr(g, field, 1)
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_gmm_window_create(8, 4, 4, g)
        assert e.value.status == fgs.FGS_ERR_UNSUPPORTED, field
    # NULL handles are refused before any device work
    for call in (lambda: fgs.fgs_eval_accumulate(0, 0, 16, fgs.FGS_MEM_HOST),
                 lambda: fgs.fgs_eval_read(0),
                 lambda: fgs.fgs_push_frame(0, 0, 0, 0, 0, fgs.FGS_MEM_HOST),
                 lambda: fgs.fgs_get_mask(0, 0, 16, fgs.FGS_MEM_HOST),
                 lambda: fgs.fgs_get_state(0)):
        with pytest.raises(fgs.FgsError) as e:
            call()
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG


def test_state_pack_unpack_roundtrip():
    import numpy as np
    from paper_2002_00250_amd import fgs
    rng = np.random.default_rng(0)
    st = dict(algo=fgs.FGS_PBAS, H=3, W=5, t=42, seed=7, N=4,
              samples=rng.integers(0, 2**32, (4, 3, 5), dtype=np.uint64).astype(np.uint32),
              dhist=rng.integers(0, 2**32, (4, 3, 5), dtype=np.uint64).astype(np.uint32),
              R=rng.random((4, 3, 5), dtype=np.float32), T=rng.random((4, 3, 5), dtype=np.float32),
              S=rng.integers(0, 9000, (4, 3, 5)).astype(np.uint16))
    back = fgs.unpack_state(fgs.pack_state(st))
    for k in ("samples", "dhist", "R", "T", "S"):
        np.testing.assert_array_equal(back[k], st[k])
    assert back["t"] == 42 and back["seed"] == 7


@pytest.mark.parametrize("diag", [False, True])
def test_gmm_state_pack_unpack_flags(diag):
    # GMM blobs: header flag bit 0 marks per-channel colour variances ([Kc][3] planes)
    import numpy as np
    from paper_2002_00250_amd import fgs
    rng = np.random.default_rng(1)
    Kc, Kd, H, W = 3, 2, 4, 6
    st = dict(algo=fgs.FGS_GMM, H=H, W=W, t=9, Kc=Kc, Kd=Kd,
              w_c=rng.random((Kc, H, W), dtype=np.float32), mu_c=rng.random((Kc, 3, H, W), dtype=np.float32),
              v_c=rng.random((Kc, 3, H, W) if diag else (Kc, H, W), dtype=np.float32),
              w_d=rng.random((Kd, H, W), dtype=np.float32), mu_d=rng.random((Kd, H, W), dtype=np.float32),
              v_d=rng.random((Kd, H, W), dtype=np.float32))
    blob = fgs.pack_state(st)
    assert blob.size == fgs.STATE_HEADER_BYTES + 4 * H * W * ((7 if diag else 5) * Kc + 3 * Kd)
    assert int(blob[28:32].view(np.int32)[0]) == (1 if diag else 0)
    back = fgs.unpack_state(blob)
    for k in ("w_c", "mu_c", "v_c", "w_d", "mu_d", "v_d"):
        np.testing.assert_array_equal(back[k], st[k])


def test_model_push_checks_tensor_arguments():
    # argument checks of the binding, before any library call (CPU tensors suffice)
    import torch
    from paper_2002_00250_amd import fgs

    class Unbound(fgs.Model):          # the checks only, no model behind them
        def __init__(self):
            self._torch, self.H, self.W = torch, 4, 6
    m = Unbound()
    bad = [(torch.zeros(4, 6, 3, dtype=torch.int16), torch.zeros(4, 6, dtype=torch.int16)),
           (torch.zeros(4, 6, 3, dtype=torch.uint8), torch.zeros(4, 6, dtype=torch.int32)),
           (torch.zeros(4, 3, 6, dtype=torch.uint8).permute(0, 2, 1), torch.zeros(4, 6, dtype=torch.int16)),
           (torch.zeros(4, 6, 3, dtype=torch.uint8), torch.zeros(6, 4, dtype=torch.int16).t()),
           (torch.zeros(5, 6, 3, dtype=torch.uint8), torch.zeros(5, 6, dtype=torch.int16))]
    for rgb, dep in bad:
        with pytest.raises(ValueError):
            m.push(rgb, dep)
    # mask read-back and ground truth: uint8 [H, W] cuda tensors with contiguous rows only
    for t in (torch.zeros(4, 6, dtype=torch.uint8), torch.zeros(6, 4, dtype=torch.uint8).t(), None):
        with pytest.raises(ValueError):
            m.mask_into(t)
        with pytest.raises(ValueError):
            m.eval_accumulate(t if t is not None else torch.zeros(4, 6, dtype=torch.int16))
