"""The largest models the library accepts (H * W = 2^28 pixels) and a PBAS image taller
than one grid dimension can index, on the launch configurations the library uses.

Frames are generated on the device (seeded).  GMM pixels are independent, so the oracle
follows sampled pixels one by one.  PBAS pixels interact through the neighbour update, so
the oracle runs windows of the image from frame 0, drawing the image's random numbers: a
window misses only the writes its outside neighbours send in, whose effect moves at most
one pixel further in per updating frame, so after u updating frames every field must equal
the GPU's at least u pixels from the window's inner edges (image edges need no margin)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from gpu_util import compare_gmm_state, log  # noqa: E402
from oracle.gmm import GmmParams, GmmRef  # noqa: E402
from oracle.pbas import PbasParams, PbasRef  # noqa: E402

MAX_PIXELS = 1 << 28


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_00250_amd import fgs
    fgs.lib()
    yield
    torch.cuda.empty_cache()


class DeviceScene:
    """Seeded frames made on the device: a fixed random background (left half at 1.5 m, right
    half at 3 m), per-frame noise, 2 % depth holes, and a moving square at 0.9 m."""

    def __init__(self, H, W, seed):
        self.H, self.W = H, W
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        self.g = g
        self.bg = torch.randint(0, 256, (H, W, 3), dtype=torch.uint8, device="cuda", generator=g)
        self.bd = torch.full((H, W), 1500, dtype=torch.int16, device="cuda")
        self.bd[:, W // 2:] = 3000
        self.side = max(4, min(H, W) // 6)

    def frame(self, t):
        H, W, g = self.H, self.W, self.g
        rgb = self.bg.to(torch.int16)
        rgb += torch.randint(-3, 4, (H, W, 3), dtype=torch.int16, device="cuda", generator=g)
        rgb = rgb.clamp_(0, 255).to(torch.uint8)
        d = self.bd + torch.randint(-10, 11, (H, W), dtype=torch.int16, device="cuda", generator=g)
        d.clamp_(min=1)
        d[torch.randint(0, 50, (H, W), dtype=torch.int16, device="cuda", generator=g) == 0] = 0
        y = (7 * t) % max(1, H - self.side)
        x = (11 * t) % max(1, W - self.side)
        rgb[y:y + self.side, x:x + self.side] = torch.tensor([200, 40, 90], dtype=torch.uint8, device="cuda")
        d[y:y + self.side, x:x + self.side] = 900
        return rgb, d


def _device_blob(m):
    from paper_2002_00250_amd import fgs
    n = fgs.fgs_state_size(m.handle)
    blob = torch.empty(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()          # the memory may still be in use on torch's stream
    fgs.fgs_copy_state(m.handle, blob.data_ptr(), n, fgs.FGS_MEM_DEVICE)
    torch.cuda.synchronize()
    return blob


def _pbas_window_state(blob, H, W, N, t, y0, x0, h, w):
    """The canonical PBAS planes of rows y0..y0+h, columns x0..x0+w, from a device blob."""
    from paper_2002_00250_amd import fgs
    n = H * W
    o = fgs.STATE_HEADER_BYTES

    def planes(off, k, dtype, npdtype):
        a = blob[off:off + k * n * np.dtype(npdtype).itemsize].view(dtype).view(k, H, W)
        return a[:, y0:y0 + h, x0:x0 + w].cpu().numpy().view(npdtype)
    st = dict(samples=planes(o, N, torch.int32, np.uint32),
              dhist=planes(o + 4 * N * n, N, torch.int32, np.uint32),
              R=planes(o + 8 * N * n, 4, torch.float32, np.float32),
              T=planes(o + 8 * N * n + 16 * n, 4, torch.float32, np.float32),
              S=planes(o + 8 * N * n + 32 * n, 4, torch.int16, np.uint16), t=t)
    return st


def _pbas_windows(H, W, N, seed, frames, windows, check_at):
    from paper_2002_00250_amd import fgs
    p = PbasParams(N=N, T_lower=1.0, T_upper=4.0, seed=seed)
    c = fgs.fgs_pbas_params_default()
    c.N, c.min_matches = p.N, p.min_matches
    c.R_incdec, c.R_scale, c.T_inc, c.T_dec = p.R_incdec, p.R_scale, p.T_inc, p.T_dec
    c.T_lower, c.T_upper = p.T_lower, p.T_upper
    for j in range(4):
        c.R_lower[j] = p.R_lower[j]
    c.depth_max_mm, c.seed = p.depth_max_mm, p.seed
    m = fgs.Model(fgs.FGS_PBAS, H, W, c)
    sc = DeviceScene(H, W, seed)
    mask = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    refs = [PbasRef(h, w, p, origin=(y0, x0, W)) for (y0, x0, h, w) in windows]
    checked = 0
    for t in range(frames):
        rgb, d = sc.frame(t)
        torch.cuda.synchronize()          # the model reads the frame on its own stream
        exps = [ref.step(rgb[y0:y0 + h, x0:x0 + w].cpu().numpy(),
                         d[y0:y0 + h, x0:x0 + w].cpu().numpy().view(np.uint16))
                for ref, (y0, x0, h, w) in zip(refs, windows)]
        m.push(rgb, d)
        if t not in check_at:
            continue
        m.mask_into(mask)
        blob = _device_blob(m)            # synchronises the device
        u = t - N + 1                     # updating frames so far
        for (y0, x0, h, w), ref, exp in zip(windows, refs, exps):
            top, left = (u if y0 > 0 else 0), (u if x0 > 0 else 0)
            bottom, right = (u if y0 + h < H else 0), (u if x0 + w < W else 0)
            inner = (slice(top, h - bottom), slice(left, w - right))
            st = _pbas_window_state(blob, H, W, N, t + 1, y0, x0, h, w)
            rs = ref.state_planes()
            bad = {k: int((np.asarray(st[k])[(Ellipsis,) + inner] != np.asarray(rs[k])[(Ellipsis,) + inner]).sum())
                   for k in ("samples", "dhist", "R", "T", "S")}
            bad["mask"] = int((mask[y0:y0 + h, x0:x0 + w].cpu().numpy()[inner] != exp[inner]).sum())
            log(f"pbas {H}x{W} N={N} t={t} window {(y0, x0, h, w)} margin {u}: {bad}")
            assert all(v == 0 for v in bad.values()), bad
            checked += 1
        del blob
        torch.cuda.synchronize()
    m.close()
    return checked


def test_pbas_max_pixels_windows():
    # 16384 x 16384 = 2^28 pixels (the limit), N = 4: the first tile, whose sample planes
    # span the full 32-bit range of a buffer resource, one in the middle, the last one.
    H = W = 16384
    assert H * W == MAX_PIXELS
    wins = [(0, 0, 16, 150), (8190, 8150, 16, 150), (H - 16, W - 150, 16, 150)]
    n = _pbas_windows(H, W, 4, 77, 7, wins, check_at=(5, 6))
    assert n == 6


def test_pbas_taller_than_grid_y():
    # 300000 rows x 70 columns: 75000 tile rows (more than a grid's y extent), ragged in x
    H, W = 300000, 70
    wins = [(0, 0, 16, 70), (150001, 0, 16, 70), (H - 16, 0, 16, 70)]
    n = _pbas_windows(H, W, 5, 31, 8, wins, check_at=(6, 7))
    assert n == 6


def test_gmm_max_pixels_sampled():
    # 2^28 pixels with the paper's Kc = 7, Kd = 3 (47 GB of state): sampled pixels, among
    # them the first and the last, follow the oracle bit for bit.
    from paper_2002_00250_amd import fgs
    H = W = 16384
    Kc, Kd = 7, 3
    p = GmmParams(Kc=Kc, Kd=Kd)
    c = fgs.fgs_gmm_params_default()
    c.Kc, c.Kd = Kc, Kd
    m = fgs.Model(fgs.FGS_GMM, H, W, c)
    sc = DeviceScene(H, W, 5)
    rng = np.random.default_rng(4)
    sel = np.unique(np.concatenate([[0, 1, W - 1, H * W - W, H * W - 1],
                                    rng.choice(H * W, 4091, replace=False)]))
    sel_d = torch.from_numpy(sel).cuda()
    ref = GmmRef(1, sel.size, p)
    mask = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    diff = total = 0
    for t in range(12):
        rgb, d = sc.frame(t)
        torch.cuda.synchronize()
        xr = rgb.view(-1, 3)[sel_d].cpu().numpy()[None]
        xd = d.view(-1)[sel_d].cpu().numpy().view(np.uint16)[None]
        exp = ref.step(xr, xd)[0]
        m.push(rgb, d)
        m.mask_into(mask)
        torch.cuda.synchronize()
        got = mask.view(-1)[sel_d].cpu().numpy()
        diff += int((got != exp).sum())
        total += sel.size
    blob = _device_blob(m)
    n = H * W
    pl = blob[fgs.STATE_HEADER_BYTES:].view(torch.float32).view(-1, n)[:, sel_d].cpu().numpy()
    del blob
    assert pl.shape[0] == 5 * Kc + 3 * Kd
    st = dict(w_c=pl[:Kc], mu_c=pl[Kc:4 * Kc].reshape(Kc, 3, -1), v_c=pl[4 * Kc:5 * Kc],
              w_d=pl[5 * Kc:5 * Kc + Kd], mu_d=pl[5 * Kc + Kd:5 * Kc + 2 * Kd],
              v_d=pl[5 * Kc + 2 * Kd:])
    refst = {k: v[..., 0, :] for k, v in ref.state_planes().items() if k != "t"}
    nv, bad, neq = compare_gmm_state(st, refst)
    log(f"gmm {H}x{W} K={Kc}/{Kd}, {sel.size} sampled px, 12 frames: mask diff {diff}/{total}, "
        f"state bad {bad}/{nv}, not bit-equal {neq}")
    m.close()
    assert diff == 0 and bad == 0 and neq == 0
