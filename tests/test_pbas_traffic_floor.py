"""The PBAS traffic-floor model: the sector counter of tests/pbas_traffic_floor.py on
hand-made cases, and the closed-form static-background floor of bench.py against that
counter on an oracle run of a static scene (every pixel background, T at its lower bound,
the regime the closed form assumes)."""
import numpy as np
import pytest

from pbas_traffic_floor import _sectors, fire_halo_bytes_per_px, step_traffic


def test_sector_count_by_hand():
    m = np.zeros((2, 32), bool)
    assert _sectors(m, 16) == 0
    m[0, 0] = m[0, 15] = True          # one sector (pixels 0..15 of row 0)
    assert _sectors(m, 16) == 1
    m[0, 16] = True                    # the next sector of that row
    m[1, 31] = True                    # the last sector of row 1
    assert _sectors(m, 16) == 3
    assert _sectors(m, 4) == 4         # pixels 0, 15, 16 of row 0 and 31 of row 1
    with pytest.raises(AssertionError):
        _sectors(np.zeros((1, 30), bool), 16)


def test_fire_halo_by_hand():
    # one 64 x 4 tile covering the image: no ring inside the image
    assert fire_halo_bytes_per_px(4, 64) == 1.0
    # 2 x 2 tiles of an 8 x 128 image: each reads 5 rows x 65 columns
    assert fire_halo_bytes_per_px(8, 128) == pytest.approx(4 * 5 * 65 / (8 * 128))
    # far from the border a tile reads 66 x 6 pixels
    assert fire_halo_bytes_per_px(400, 640) == pytest.approx(66 * 6 / 256, rel=0.03)


@pytest.fixture(scope="module")
def static_counts():
    from oracle.pbas import PbasParams, PbasRef
    from synth import Scene, SceneConfig
    H, W, N = 64, 256, 35
    sc = Scene(SceneConfig(H=H, W=W, n_objects=0))
    ref = PbasRef(H, W, PbasParams(N=N))
    for t in range(N + 6):
        rgb, D, _ = sc.frame(t)
        ref.step(rgb, D)
    acc, fg, T_low = [], [], []
    for t in range(N + 6, N + 10):
        rgb, D, _ = sc.frame(t)
        T_low.append(float((ref.T == np.float32(2.0)).mean()))
        acc.append(step_traffic(ref, rgb, D))
        fg.append(float(ref.last_F.any(-1).mean()))
    return acc, fg, T_low


def test_static_scene_is_the_closed_forms_regime(static_counts):
    _, fg, T_low = static_counts
    assert max(fg) < 0.002 and min(T_low) > 0.999


def test_closed_form_matches_oracle_count_on_static_scene(static_counts):
    import bench
    acc, _, _ = static_counts
    for g in (64, 128):
        # 2 % of the pixels have no depth: 3.98 active channels on average
        cf = bench.pbas_static_floor_bytes_per_px(N=35, T=2.0, channels=3.98, gran=g, H=64, W=256)
        d_read = np.mean([a[g]["D_read"] for a in acc])
        landed = np.mean([a[g]["samples_landed"] for a in acc])
        changed = np.mean([a[g]["samples_write"] for a in acc])
        # D reads: the same events (self-updates at uniform slots)
        assert d_read == pytest.approx(cf["D_read"], rel=0.03), (g, d_read, cf["D_read"])
        # sample sectors an update lands in: the closed form's events; the top and bottom
        # rows receive fewer neighbour writes, so the count sits slightly below it
        assert 0.98 * cf["samples_write"] < landed <= cf["samples_write"] * 1.005, (g, landed, cf)
        # sectors whose bytes change are a subset (a write may store the byte it replaces)
        assert changed <= landed
