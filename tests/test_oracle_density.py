"""Pins of the oracle's densification, pruning and opacity reset (3DGS's density
control, which the paper keeps for its first phase: Sec. 5.1 "Implementation
Details").  Each test checks the oracle against a closed form or a hand-derived
outcome, not against its own code."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_13855_amd import scenes
from tests.test_oracle_pins import axis_camera, iso_alpha, set_splat, sigmoid, splats

RULES = O.DensityRules(grad_threshold=1e-3, percent_dense=0.01, scene_extent=10.0, min_opacity=0.005,
                       max_screen_size=20.0, max_world_frac=0.5, keep_probability=0.5)


def test_statistic_single_splat_closed_form():
    """One isotropic splat: C = c0 + alpha (c - c0), so dL/dmx = sum g (c - c0) alpha dx / var;
    the statistic is |(dL/dmx W/2, dL/dmy H/2)|, counted once, radius 3 sqrt(var)."""
    cam = axis_camera()
    bg = np.array([0.1, 0.2, 0.3])
    c = np.array([0.8, 0.3, 0.6])
    p = splats(1)
    s, logit = 0.05, 0.5
    set_splat(p, 0, (0.0, 0.0, 0.0), s, logit=logit, color=c, v=0.7)     # on the axis: isotropic on screen
    rng = np.random.default_rng(5)
    g = rng.normal(size=(3, cam.height, cam.width))
    acc, den, rad = O.densify_stats(p, 10.0, bg, [cam], [g])
    z = 3.0
    mx, my = cam.cx, cam.cy
    var = (cam.fx * s / z) ** 2 + 0.3
    a = iso_alpha(cam, sigmoid(logit), s, z, mx, my)
    a = np.where(a >= 1 / 255, a, 0.0)
    X, Y = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5)
    w = (g * (c - bg)[:, None, None]).sum(axis=0) * a / var
    gx, gy = (w * (X - mx)).sum(), (w * (Y - my)).sum()
    assert acc[0] == pytest.approx(math.hypot(gx * cam.width / 2, gy * cam.height / 2), rel=1e-9)
    assert den[0] == 1.0
    assert rad[0] == pytest.approx(3.0 * math.sqrt(var), rel=1e-12)


def test_statistic_counts_visible_views_only():
    """A view that has the splat behind it, and one where its footprint lies beside the
    image, add nothing; the statistic accumulates over the views that see it."""
    front = axis_camera()
    behind = scenes.look_at_camera((0.0, 0.0, 3.0), 64, 48, target=(0.0, 0.0, 6.0))
    p = splats(2)
    set_splat(p, 0, (0.0, 0.0, 0.0), 0.05, logit=0.5)
    set_splat(p, 1, (3.0, 0.0, 0.0), 0.01, logit=0.5)     # projects far right of the image
    rng = np.random.default_rng(6)
    g = [rng.normal(size=(3, 48, 64)) for _ in range(3)]
    acc1, den1, _ = O.densify_stats(p, 10.0, np.zeros(3), [front], [g[0]])
    acc3, den3, _ = O.densify_stats(p, 10.0, np.zeros(3), [front, behind, front], [g[0], g[1], g[2]])
    acc_g2, _, _ = O.densify_stats(p, 10.0, np.zeros(3), [front], [g[2]])
    assert den1[0] == 1 and den3[0] == 2
    assert acc3[0] == pytest.approx(acc1[0] + acc_g2[0], rel=1e-12)
    assert den1[1] == 0 and den3[1] == 0 and acc3[1] == 0.0


def test_split_children_lie_on_the_rotated_axes():
    """A quarter turn about z maps the x axis to y: the child drawn at z = e_x sits at
    mean + s_x e_y, the one at -e_z at mean - s_z e_z; scales are divided by 1.6."""
    p = splats(1)
    h = math.sqrt(0.5)
    set_splat(p, 0, (0.3, -0.2, 0.1), (0.2, 0.05, 0.1), quat=(h, 0.0, 0.0, h))
    c1 = O.split_child(p, 0, (1.0, 0.0, 0.0))
    c2 = O.split_child(p, 0, (0.0, 0.0, -1.0))
    np.testing.assert_allclose(c1["mean"], [0.3, -0.2 + 0.2, 0.1], atol=1e-15)
    np.testing.assert_allclose(c2["mean"], [0.3, -0.2, 0.1 - 0.1], atol=1e-15)
    np.testing.assert_allclose(np.exp(c1["log_scale"]), np.array([0.2, 0.05, 0.1]) / 1.6, rtol=1e-14)
    for g in ("quat", "opacity_logit", "sh", "vsh"):
        np.testing.assert_array_equal(c1[g], p[g][:, 0])


def hand_set():
    """Eleven splats, one per case (statistic = accum / denom, extent 10 => clone when
    max scale <= 0.1; world limit 0.5 x 10 = 5; screen limit 20 px):
      0 not a candidate, kept            1 candidate, small, drawn in -> cloned
      2 candidate, large -> split        3 opacity below the minimum -> pruned
      4 candidate, small, low opacity -> original and copy pruned
      5 candidate, large -> split        6 original too large on screen -> pruned
      7 candidate by gradient, drawn out (u >= p) -> kept as it is
      8 candidate, small, too large on screen -> original pruned, its copy kept
      9 sum above the threshold, mean (sum / 3 views) below -> kept as it is
     10 candidate with largest scale 6 > 5 -> split; children (6 / 1.6) kept"""
    p = splats(11)
    for i in range(11):
        set_splat(p, i, (0.1 * i, 0.0, 0.0), 0.05, logit=0.0)
    for i in (2, 5):
        p["log_scale"][:, i] = np.log([0.3, 0.1, 0.1])
    p["log_scale"][:, 10] = np.log([6.0, 0.1, 0.1])
    p["opacity_logit"][0, 3] = -7.0
    p["opacity_logit"][0, 4] = -7.0
    accum = np.array([1e-4, 5e-3, 6e-3, 0, 4e-3, 2e-3, 0, 9e-3, 4e-3, 2.4e-3, 2e-3])
    denom = np.array([1, 2, 2, 1, 1, 1, 1, 3, 1, 3, 1], float)
    radius = np.array([5, 5, 5, 5, 5, 5, 25, 5, 25, 5, 5], float)
    uniform = np.array([0.9, 0.3, 0.1, 0.2, 0.4, 0.49, 0.1, 0.7, 0.3, 0.1, 0.2])
    return p, accum, denom, radius, uniform


def test_densify_hand_case_order_and_moments():
    p, accum, denom, radius, uniform = hand_set()
    rng = np.random.default_rng(7)
    m = {g: rng.normal(size=(c, 11)) for g, c in O.GROUPS}
    v = {g: rng.random(size=(c, 11)) for g, c in O.GROUPS}
    normals = rng.normal(size=(11, 2, 3))
    q, qm, qv, src = O.densify(p, m, v, accum, denom, radius, uniform, normals, RULES)
    # originals 0, 1, 7, 9; clones of 1, 8; first children of 2, 5, 10; second children
    np.testing.assert_array_equal(src, [0, 1, 7, 9, 1, 8, 2, 5, 10, 2, 5, 10])
    for j, i in enumerate([0, 1, 7, 9]):
        for g, _ in O.GROUPS:
            np.testing.assert_array_equal(q[g][:, j], p[g][:, i])
            np.testing.assert_array_equal(qm[g][:, j], m[g][:, i])
            np.testing.assert_array_equal(qv[g][:, j], v[g][:, i])
    for j in range(4, 12):
        for g, _ in O.GROUPS:
            assert not qm[g][:, j].any() and not qv[g][:, j].any()
    for g, _ in O.GROUPS:
        np.testing.assert_array_equal(q[g][:, 4], p[g][:, 1])
        np.testing.assert_array_equal(q[g][:, 5], p[g][:, 8])
    for j, (i, k) in zip(range(6, 12), [(2, 0), (5, 0), (10, 0), (2, 1), (5, 1), (10, 1)]):
        ch = O.split_child(p, i, normals[i][k])
        for g, _ in O.GROUPS:
            np.testing.assert_array_equal(q[g][:, j], ch[g])


def test_keep_probability_extremes_and_count():
    p, accum, denom, radius, uniform = hand_set()
    zeros = {g: np.zeros((c, 11)) for g, c in O.GROUPS}
    normals = np.zeros((11, 2, 3))
    # p = 0: nothing densifies (10 is then an original beyond the world limit: pruned);
    # p = 1: 7 (mean 3e-3, small) is cloned as well
    for prob, want in ((0.0, [0, 1, 2, 5, 7, 9]), (1.0, [0, 1, 7, 9, 1, 7, 8, 2, 5, 10, 2, 5, 10])):
        r = O.DensityRules(**{**RULES.__dict__, "keep_probability": prob})
        _, _, _, src = O.densify(p, zeros, zeros, accum, denom, radius, uniform, normals, r)
        np.testing.assert_array_equal(src, want)
    clone, split, ko, kc, kch = O.densify_decisions(p, accum, denom, radius, uniform, RULES)
    _, _, _, src = O.densify(p, zeros, zeros, accum, denom, radius, uniform, normals, RULES)
    assert len(src) == ko.sum() + kc.sum() + 2 * kch.sum()
    # the draw u ~ U[0, 1) keeps a candidate iff u < p: a draw of exactly 0 with p = 0 and a
    # draw equal to p are not kept (p = 0 never densifies, p = 1 always does)
    for prob in (0.0, float(uniform[7])):
        u = uniform.copy()
        u[7] = prob
        r = O.DensityRules(**{**RULES.__dict__, "keep_probability": prob})
        clone, split, _, _, _ = O.densify_decisions(p, accum, denom, radius, u, r)
        assert not clone[7] and not split[7]


def test_reset_opacity_clamps_and_restarts_moments():
    p = splats(3)
    p["opacity_logit"][0] = [2.0, -3.0, -6.0]
    m = {g: np.ones((c, 3)) for g, c in O.GROUPS}
    v = {g: np.ones((c, 3)) for g, c in O.GROUPS}
    O.reset_opacity(p, m, v, 0.01)
    o = 1.0 / (1.0 + np.exp(-p["opacity_logit"][0]))
    np.testing.assert_allclose(o[:2], [0.01, 0.01], rtol=1e-12)
    assert p["opacity_logit"][0, 2] == -6.0
    assert not m["opacity_logit"].any() and not v["opacity_logit"].any()
    assert m["mean"].all() and v["sh"].all()
