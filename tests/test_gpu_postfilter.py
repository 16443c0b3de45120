"""Median post-filter of a binary mask on the GPU against the oracle: ragged sizes around
the 256 x 16 tile at every radius, strided buffers with guard bytes, empty images, a
model's own 1280x720 mask, a tall image and the largest model size (sampled row bands),
and the argument checks."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import log  # noqa: E402
from oracle.postfilter import median_mask as oracle_median  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield
    torch.cuda.empty_cache()


def _mask(H, W, seed, kind):
    rng = np.random.default_rng(seed)
    if kind == "noise":
        return np.where(rng.random((H, W)) < 0.5, 255, 0).astype(np.uint8)
    if kind == "values":            # any nonzero byte is foreground
        return (rng.integers(0, 2, (H, W)) * rng.integers(1, 256, (H, W))).astype(np.uint8)
    # blobs: a smooth random field thresholded, with salt-and-pepper noise
    f = rng.standard_normal((H // 8 + 2, W // 8 + 2))
    f = np.kron(f, np.ones((8, 8)))[:H, :W]
    m = f > 0.2
    m ^= rng.random((H, W)) < 0.05
    return np.where(m, 255, 0).astype(np.uint8)


def _gpu_median(m, r, src_pad=0, dst_pad=0):
    """Filter host mask m on the device; rows padded by guard bytes that must stay as set."""
    from paper_2002_00250_amd import fgs
    H, W = m.shape
    src = torch.full((H, W + src_pad), 3, dtype=torch.uint8, device="cuda")
    src[:, :W] = torch.from_numpy(m).cuda()
    dst = torch.full((H, W + dst_pad), 77, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    fgs.fgs_mask_median(src.data_ptr(), W + src_pad, dst.data_ptr(), W + dst_pad, H, W, r,
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    out = dst.cpu().numpy()
    assert (out[:, W:] == 77).all(), "guard bytes written"
    return out[:, :W]


SHAPES = [(1, 1), (1, 300), (300, 1), (16, 256), (17, 257), (15, 255), (33, 513), (250, 700)]


@pytest.mark.parametrize("H,W", SHAPES)
def test_parity_every_radius(H, W):
    for r in range(8):
        for kind in ("noise", "values", "blobs"):
            m = _mask(H, W, 1000 * r + H + W, kind)
            got = _gpu_median(m, r)
            bad = int((got != oracle_median(m, r)).sum())
            assert bad == 0, (H, W, r, kind, bad)
    log(f"median {H}x{W}: radii 0..7, 3 mask kinds equal")


def test_strided_buffers():
    m = _mask(45, 300, 7, "blobs")
    for r in (1, 4, 7):
        got = _gpu_median(m, r, src_pad=61, dst_pad=13)
        assert np.array_equal(got, oracle_median(m, r)), r


def test_empty_images():
    from paper_2002_00250_amd import fgs
    fgs.fgs_mask_median(0, 0, 0, 0, 0, 5, 3)
    fgs.fgs_mask_median(0, 0, 0, 0, 7, 0, 3)
    e = torch.empty((0, 9), dtype=torch.uint8, device="cuda")
    assert fgs.median_mask(e, 2).shape == (0, 9)


def test_model_mask_720p():
    # a GMM K=5 model's own 1280x720 mask, filtered on the device on torch's stream through
    # the binding at the base method's 9x9 window and the largest; the oracle filters the
    # oracle model's mask of the same frames, which the device mask must equal first
    from paper_2002_00250_amd import fgs
    from oracle.gmm import GmmParams, GmmRef
    from synth import Scene, preset
    sc = Scene(preset("hd_1280x720"))
    gp = fgs.fgs_gmm_params_default()
    gp.Kc, gp.Kd = 5, 5
    m = fgs.Model(fgs.FGS_GMM, 720, 1280, gp)
    ref = GmmRef(720, 1280, GmmParams(Kc=5, Kd=5))
    for t in range(12):
        rgb, d, _ = sc.frame(t)
        m.push(rgb, d)
        ref_mask = ref.step(rgb, d)
    dm = torch.empty((720, 1280), dtype=torch.uint8, device="cuda")
    m.mask_into(dm)
    torch.cuda.synchronize()
    assert np.array_equal(dm.cpu().numpy(), ref_mask)
    fg = float((ref_mask != 0).mean())
    for r in (4, 7):
        out = fgs.median_mask(dm, r)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        bad = int((got != oracle_median(ref_mask, r)).sum())
        log(f"median 720p model mask r={r}: foreground {fg:.3f} -> {float((got != 0).mean()):.3f}, diff {bad}")
        assert bad == 0
    m.close()


@pytest.mark.parametrize("H,W,r", [(70000, 70, 7), (16384, 16384, 7)])
def test_large_images_sampled_bands(H, W, r):
    # every output row of a band depends only on rows within r of it, so the oracle filters
    # the bands (first, middle, last) from the whole image
    from paper_2002_00250_amd import fgs
    g = torch.Generator(device="cuda")
    g.manual_seed(H + W)
    src = (torch.rand((H, W), device="cuda", generator=g) < 0.5).to(torch.uint8) * 255
    dst = torch.full((H, W), 77, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    fgs.fgs_mask_median(src.data_ptr(), W, dst.data_ptr(), W, H, W, r, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    host = src.cpu().numpy()
    for y0 in (0, H // 2 - 20, H - 40):
        band = slice(y0, y0 + 40)
        got = dst[band].cpu().numpy()
        bad = int((got != oracle_median(host, r, rows=band)).sum())
        log(f"median {H}x{W} r={r} rows {y0}..{y0 + 40}: diff {bad}")
        assert bad == 0
    del src, dst


def test_argument_checks():
    from paper_2002_00250_amd import fgs
    a = torch.zeros((8, 40), dtype=torch.uint8, device="cuda")
    b = torch.zeros((8, 40), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    bad = [
        (a.data_ptr(), 40, b.data_ptr(), 40, 8, 40, 8),       # radius above 7
        (a.data_ptr(), 40, b.data_ptr(), 40, 8, 40, -1),      # negative radius
        (a.data_ptr(), 39, b.data_ptr(), 40, 8, 40, 1),       # source stride below W
        (a.data_ptr(), 40, b.data_ptr(), 39, 8, 40, 1),       # destination stride below W
        (a.data_ptr(), 40, b.data_ptr(), 40, -1, 40, 1),      # negative height
        (a.data_ptr(), 40, b.data_ptr(), 40, 8, (1 << 30) + 1, 1),  # width above 2^30
        (0, 40, b.data_ptr(), 40, 8, 40, 1),                  # NULL source
        (a.data_ptr(), 40, a.data_ptr() + 40, 40, 7, 40, 1),  # overlapping rows
        (a.data_ptr(), 40, a.data_ptr(), 40, 8, 40, 1),       # in place
    ]
    for args in bad:
        with pytest.raises(fgs.FgsError) as e:
            fgs.fgs_mask_median(*args)
        assert e.value.status == fgs.FGS_ERR_INVALID_ARG, args
    with pytest.raises(ValueError):
        fgs.median_mask(a.float(), 1)
    with pytest.raises(ValueError):
        fgs.median_mask(a, 1, out=torch.zeros((8, 41), dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):   # rows broadcast from one: a row stride of 0
        fgs.median_mask(a[:1].expand(8, 40), 1)
    # a row-strided view (every other row of a taller buffer) is filtered as laid out
    tall = torch.from_numpy(_mask(16, 40, 3, "noise")).cuda()
    got = fgs.median_mask(tall[::2], 2)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle_median(tall[::2].cpu().numpy(), 2))
    # the buffers were never written
    torch.cuda.synchronize()
    assert int(b.sum()) == 0
