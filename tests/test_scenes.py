"""The seeded input generator: shapes, determinism and camera geometry (CPU)."""
import math

import numpy as np

from paper_2605_13855_amd import scenes


def test_config_shapes_and_determinism():
    a = scenes.make_scene(1)
    b = scenes.make_scene(1)
    assert a.n == 2000 and len(a.cameras) == 1 and a.cameras[0].width == 128
    for g, c in scenes.PARAM_GROUPS:
        assert a.params[g].shape == (c, 2000) and a.params[g].dtype == np.float32
        assert np.array_equal(a.params[g], b.params[g])
    assert np.array_equal(a.targets[0], b.targets[0])
    q = a.params["quat"].astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(q, axis=0), 1.0, atol=1e-6)
    assert abs(float(a.params["vsh"][0].mean()) - 1.0) < 0.05


def test_batched_views_are_uneven_and_on_the_orbit():
    sc = scenes.make_scene(4, n=1000)
    assert len(sc.cameras) == 16
    ws = {c.width for c in sc.cameras}
    assert len(ws) > 8 and min(ws) >= 640 and max(ws) <= 1600
    for c in sc.cameras:
        assert c.height == int(round(0.75 * c.width))
        assert np.linalg.norm(c.center()) == np.float64(np.linalg.norm(c.center()))
        assert abs(np.linalg.norm(c.center()) - 4.0) < 1e-4
        # the origin projects to the image centre
        pc = np.asarray(c.R, np.float64) @ np.zeros(3) + np.asarray(c.t, np.float64)
        assert abs(c.fx * pc[0] / pc[2] + c.cx - c.width / 2) < 1e-3


def test_look_at_camera_is_a_rotation_with_horizontal_fov():
    c = scenes.orbit_camera(3.0, 0.7, -0.2, 200, 100)
    R = np.asarray(c.R, np.float64)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-6)
    assert abs(np.linalg.det(R) - 1.0) < 1e-6
    assert abs(2 * math.degrees(math.atan(c.width / (2 * c.fx))) - 60.0) < 1e-9


def test_cluster_scene_is_clustered():
    sc = scenes.make_scene(5, n=20000, width=64, height=36)
    m = sc.params["mean"].astype(np.float64)
    assert m.shape == (3, 20000)
    # tighter nearest-neighbour spacing than a uniform cube [-2, 2]^3 of the same count
    def nn_median(pts):
        d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
        np.fill_diagonal(d, np.inf)
        return float(np.median(d.min(axis=1)))

    uni = np.random.default_rng(0).uniform(-2, 2, size=(2000, 3))
    assert nn_median(m[:, :2000].T) < 0.85 * nn_median(uni)
