"""Seeded generators: byte-identical reproduction and the stated statistics."""
import numpy as np

import scenegen


def test_seeds_reproduce_bytes():
    a = scenegen.tiny_scene()
    b = scenegen.tiny_scene()
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "mask_scores", "masks"):
        assert a[k].tobytes() == b[k].tobytes()
    assert a["targets"][0].tobytes() == b["targets"][0].tobytes()


def test_tiny_scene_statistics():
    s = scenegen.tiny_scene()
    assert s["means"].shape == (4096, 3) and s["sh"].shape == (4096, 1, 3)
    assert np.all(np.abs(s["means"]) <= 1.0)
    assert abs(s["log_scales"].mean() + 3.0) < 0.02 and abs(s["log_scales"].std() - 0.3) < 0.02
    np.testing.assert_allclose(np.linalg.norm(s["quats"], axis=1), 1.0, atol=1e-6)
    p = 1 / (1 + np.exp(-s["mask_scores"][:, 0]))
    assert abs(s["masks"].mean() - p.mean()) < 0.03
    cam = s["cameras"][0]
    np.testing.assert_allclose(cam["viewmat"], np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 4], [0, 0, 0, 1]]),
                               atol=1e-6)
    assert abs(float(cam["fx"]) - 64 / np.tan(np.radians(30))) < 1e-3


def test_object_scene_inside_unit_ball():
    s = scenegen.object_scene(n=6400, width=64, height=64)
    assert np.all(np.linalg.norm(s["means"].astype(np.float64), axis=1) <= 1.0 + 1e-6)
    assert s["sh"].shape == (6400, 16, 3)


def test_unbounded_scene_shell_and_tails():
    s = scenegen.unbounded_scene(n=64_000, width=64, height=64)
    r = np.linalg.norm(s["means"].astype(np.float64), axis=1)
    fg = r <= 3.0 + 1e-6
    assert abs(fg.mean() - 0.8) < 0.01
    assert np.all((r[~fg] >= 20.0 - 1e-4) & (r[~fg] <= 50.0 + 1e-4))
    ls = s["log_scales"].astype(np.float64)
    assert ls.max() <= scenegen.LOG_SCALE_CAP + 1e-6
    # Student-t(3) tail: P(t > 5) ~ 0.0077 -> log-scale above 0 for ~0.77% of axes
    frac = (ls > 0).mean()
    assert 0.004 < frac < 0.012


def test_orbit_camera_looks_at_origin():
    cam = scenegen.orbit_camera(5.0, 45.0, 15.0, 100, 80)
    vm = cam["viewmat"].astype(np.float64)
    t = vm[:3, :3] @ np.zeros(3) + vm[:3, 3]
    assert abs(t[0]) < 1e-5 and abs(t[1]) < 1e-5 and abs(t[2] - 5.0) < 1e-5
    np.testing.assert_allclose(vm[:3, :3] @ vm[:3, :3].T, np.eye(3), atol=1e-6)
    assert abs(np.linalg.det(vm[:3, :3]) - 1.0) < 1e-6
