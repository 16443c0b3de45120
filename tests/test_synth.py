"""The synthetic scene generator: deterministic per (config, t), shapes, ranges and the
statistics its docstring promises."""
import numpy as np

from synth import Scene, preset


def test_frame_is_pure_function_of_config_and_t():
    cfg = preset("gmm_320x240")
    a, b = Scene(cfg), Scene(cfg)
    for t in (0, 7, 3):
        for x, y in zip(a.frame(t), b.frame(t)):
            np.testing.assert_array_equal(x, y)
    assert not np.array_equal(a.frame(1)[0], a.frame(2)[0])


def test_shapes_types_and_holes():
    for name in ("gmm_320x240", "pbas_640x480"):
        cfg = preset(name)
        rgb, d, gt = Scene(cfg).frame(3)
        assert rgb.shape == (cfg.H, cfg.W, 3) and rgb.dtype == np.uint8
        assert d.shape == (cfg.H, cfg.W) and d.dtype == np.uint16
        assert gt.dtype == np.uint8 and set(np.unique(gt)) <= {0, 255}
        assert 0.015 < (d == 0).mean() < 0.025
        v = d[(d > 0) & (gt == 0)]
        assert abs(np.median(v[v < 2000]) - 1500) < 5 and abs(np.median(v[v > 2000]) - 3000) < 5


def test_noise_free_static_scene_is_constant():
    cfg = preset("gmm_320x240", n_objects=0, rgb_noise=0.0, depth_noise_mm=0.0, hole_frac=0.0)
    s = Scene(cfg)
    for x, y in zip(s.frame(0), s.frame(50)):
        np.testing.assert_array_equal(x, y)


def test_camouflage_object_changes_depth_only():
    cfg = preset("pbas_640x480", n_objects=0, illumination=False, rgb_noise=0.0,
                 depth_noise_mm=0.0, hole_frac=0.0)
    s = Scene(cfg)
    rgb, d, gt = s.frame(10)
    np.testing.assert_array_equal(rgb, np.clip(s.bg_rgb, 0, 255).astype(np.uint8))
    obj = gt == 255
    assert obj.any()
    np.testing.assert_array_equal(d[obj].astype(int), s.bg_depth[obj].astype(int) - 600)
