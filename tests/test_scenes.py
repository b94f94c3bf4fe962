"""The seeded input generator: shapes, value ranges and analytic depths."""

import math

import numpy as np

import scenes


def test_c1_shapes_ranges_and_seed():
    a = scenes.make_scene("c1")
    b = scenes.make_scene("c1")
    assert a.depth.shape == (128, 128) and a.normal_rough.shape == (128, 128, 4)
    assert a.env.shape == (32, 64, 3)
    for k in ("depth", "normal_rough", "albedo_metal", "radiance", "env"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
        assert getattr(a, k).dtype == np.float32 and getattr(a, k).flags.c_contiguous
    fg = np.isfinite(a.depth)
    assert 0.1 < fg.mean() < 1.0
    n = a.normal_rough[fg, :3]
    assert np.abs(np.linalg.norm(n, axis=1) - 1).max() < 1e-6
    r = a.normal_rough[fg, 3]
    assert r.min() >= 0.05 and r.max() <= 1.0
    assert set(np.unique(a.albedo_metal[fg, 3])) <= {0.0, 1.0}
    assert np.all(a.radiance[~fg] == 0) and np.all(a.normal_rough[~fg] == 0)


def test_floor_depth_is_analytic():
    """Pixels that see the ground plane have the plane's exact view depth."""
    s = scenes.make_scene("c1")
    c = s.camera
    rot = c["rot"].astype(np.float64)
    h, w = s.depth.shape
    floor = np.isfinite(s.depth) & (np.abs(s.normal_rough[..., 1] - 1) < 1e-7)
    jj, ii = np.nonzero(floor)
    x = (ii + 0.5 - float(c["cx"])) / float(c["fx"])
    y = -(jj + 0.5 - float(c["cy"])) / float(c["fy"])
    d = x[:, None] * rot[0] + y[:, None] * rot[1] + rot[2]
    t = -float(c["pos"][1]) / d[:, 1]
    z = (t[:, None] * d) @ rot[2]
    assert np.allclose(s.depth[floor], z, rtol=1e-6)


def test_headline_scene_and_quantisation():
    s = scenes.make_scene("c2", width=192, height=108)
    assert s.params["spp"] == 16 and s.params["march"] == 1 and s.env.shape == (256, 512, 3)
    lg = np.log(s.env)
    assert abs(lg.mean()) < 0.05 and abs(lg.std() - 2.0) < 0.05
    bits, vals = scenes.quantise_gbuffer(s, "f16")
    assert np.array_equal(vals["albedo_metal"], s.albedo_metal.astype(np.float16).astype(np.float32))
    bits, vals = scenes.quantise_gbuffer(s, "bf16")
    x = s.normal_rough
    rel = np.abs(vals["normal_rough"] - x) / np.maximum(np.abs(x), 1e-30)
    assert rel[np.abs(x) > 1e-30].max() <= 2 ** -8
    # round-to-nearest-even on a tie: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6 (even)
    t = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8], np.float32)
    assert np.array_equal(scenes.bf16_round(t), np.array([0x3F80, 0x3F82], np.uint16))


def test_camera_is_look_at():
    c = scenes.look_at_camera(1920, 1080, (0, 1.5, 5), (0, 0, 0), 60.0, 0.01)
    assert abs(float(c["fy"]) - 540 / math.tan(math.radians(30))) < 1e-3
    f = c["rot"][2].astype(np.float64)
    assert np.allclose(f, -np.array([0, 1.5, 5]) / np.linalg.norm([0, 1.5, 5]), atol=1e-7)
