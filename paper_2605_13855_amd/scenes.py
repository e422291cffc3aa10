"""Seeded synthetic scenes and cameras.

This module only draws inputs: splat parameters in the component-major layout the
renderer takes, look-at pinhole cameras and target images. It holds none of the
renderer's arithmetic (no projection, colour or blending), so it is the one module
that both the FP64 oracle tests and the GPU path consume.

Every draw uses ``numpy.random.Generator(PCG64(seed))`` in a fixed order:
means, log-scales, quaternions, opacity logits, colour SH, view-weight SH, targets,
cameras.  The distributions follow the workloads the paper trains on (a few hundred
thousand to a few million anisotropic splats of a few pixels, degree-3 SH colour,
a single-channel degree-3 SH view weight), in the shapes the five benchmark
configurations fix:

* log-scale ~ N(-3.5, 0.3), quaternion = normalised N(0, I4), opacity logit ~ N(0, 1)
* colour SH ~ N(0, 0.2) (16 x 3), view-weight SH ~ N(0, 0.2) (16) with +1 on its DC term
* sigma = 10, black background, target ~ U[0, 1]^(3HW), horizontal fov 60 degrees
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Parameter groups and their component counts; layout is [C][N] float32 each.
PARAM_GROUPS = (
    ("mean", 3),
    ("log_scale", 3),
    ("quat", 4),            # (w, x, y, z), not necessarily unit length
    ("opacity_logit", 1),
    ("sh", 48),             # [16 coefficients][3 channels]
    ("vsh", 16),            # single-channel view-weight SH
)
N_COMPONENTS = sum(c for _, c in PARAM_GROUPS)  # 75


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV convention (+x right, +y down, +z forward).

    ``R`` (3x3, row-major) and ``t`` map world to camera: x_cam = R x_world + t.
    Pixel (i, j) has its centre at (i + 0.5, j + 0.5).
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray
    t: np.ndarray
    near: float = 0.2

    def center(self) -> np.ndarray:
        return -np.asarray(self.R, np.float64).T @ np.asarray(self.t, np.float64)


@dataclasses.dataclass
class Scene:
    params: dict          # name -> float32 array [C][N] (opacity_logit is [1][N])
    sigma: float
    background: np.ndarray  # float32 [3]
    cameras: list
    targets: list         # float32 [3][H][W] per camera

    @property
    def n(self) -> int:
        return int(self.params["mean"].shape[1])


def look_at_camera(center, width, height, fov_x_deg=60.0, target=(0.0, 0.0, 0.0)):
    """Camera at ``center`` whose +z axis points at ``target``; world +y is image down."""
    center = np.asarray(center, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - center
    fwd /= np.linalg.norm(fwd)
    down = np.array([0.0, 1.0, 0.0])
    right = np.cross(down, fwd)
    if np.linalg.norm(right) < 1e-9:          # looking straight up or down
        right = np.array([1.0, 0.0, 0.0])
    right /= np.linalg.norm(right)
    dn = np.cross(fwd, right)
    R = np.stack([right, dn, fwd]).astype(np.float32)
    t = (-R.astype(np.float64) @ center).astype(np.float32)
    fx = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    return Camera(width=int(width), height=int(height), fx=float(fx), fy=float(fx),
                  cx=width / 2.0, cy=height / 2.0, R=R, t=t)


def orbit_camera(radius, azimuth, elevation, width, height, fov_x_deg=60.0):
    """Camera on a sphere of ``radius`` around the origin, looking at the origin.

    azimuth 0 / elevation 0 is the point (0, 0, -radius); positive elevation is up (-y).
    """
    c = (radius * math.sin(azimuth) * math.cos(elevation),
         -radius * math.sin(elevation),
         -radius * math.cos(azimuth) * math.cos(elevation))
    return look_at_camera(c, width, height, fov_x_deg)


def _draw_splats(rng, n, mean_lo, mean_hi, log_scale_mu=-3.5, log_scale_sd=0.3, means=None):
    if means is None:
        mean = rng.uniform(mean_lo, mean_hi, size=(3, n))
    else:
        mean = means
    log_scale = rng.normal(log_scale_mu, log_scale_sd, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity_logit = rng.normal(0.0, 1.0, size=(1, n))
    sh = rng.normal(0.0, 0.2, size=(48, n))
    vsh = rng.normal(0.0, 0.2, size=(16, n))
    vsh[0] += 1.0
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return {"mean": f32(mean), "log_scale": f32(log_scale), "quat": f32(q),
            "opacity_logit": f32(opacity_logit), "sh": f32(sh), "vsh": f32(vsh)}


def _targets(rng, cams):
    return [rng.uniform(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cams]


def _cluster_means(rng, n, n_clusters=64):
    centres = rng.uniform(-2.0, 2.0, size=(n_clusters, 3))
    stds = rng.uniform(0.05, 0.5, size=(n_clusters, 3))
    rots = []
    for _ in range(n_clusters):
        a = rng.normal(size=(3, 3))
        qm, r = np.linalg.qr(a)
        qm *= np.sign(np.diag(r))[None, :]
        rots.append(qm)
    which = rng.integers(0, n_clusters, size=n)
    local = rng.normal(size=(n, 3)) * stds[which]
    rots = np.stack(rots)
    pts = np.einsum("nij,nj->ni", rots[which], local) + centres[which]
    return np.ascontiguousarray(pts.T)


def make_scene(config: int, seed: int | None = None, n: int | None = None,
               width: int | None = None, height: int | None = None,
               log_scale_mu: float = -3.5) -> Scene:
    """Build one of the five benchmark workloads (optionally shrunk for tests).

    1: 2,000 splats in [-1,1]^3, one 128x128 view from distance 3.
    2: 100,000 splats in [-2,2]^3, one 800x800 view from distance 3.
    3: 500,000 splats in [-2,2]^3, one 1600x1064 view from distance 3.
    4: 1,000,000 splats in [-2,2]^3, 16 views of uneven size (640x480 .. 1600x1200)
       on an orbit of radius 4.
    5: 3,000,000 splats from 64 anisotropic clusters, 8 views 1960x1090 on the orbit.
    """
    if seed is None:
        seed = config
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = {
        1: dict(n=2000, lo=-1.0, hi=1.0, w=128, h=128),
        2: dict(n=100_000, lo=-2.0, hi=2.0, w=800, h=800),
        3: dict(n=500_000, lo=-2.0, hi=2.0, w=1600, h=1064),
        4: dict(n=1_000_000, lo=-2.0, hi=2.0),
        5: dict(n=3_000_000, lo=-2.0, hi=2.0),
    }[config]
    nn = n if n is not None else spec["n"]
    if config == 5:
        means = _cluster_means(rng, nn)
        params = _draw_splats(rng, nn, 0, 0, log_scale_mu=log_scale_mu, means=means)
    else:
        params = _draw_splats(rng, nn, spec["lo"], spec["hi"], log_scale_mu=log_scale_mu)
    if config in (1, 2, 3):
        w = width if width is not None else spec["w"]
        h = height if height is not None else spec["h"]
        cams = [look_at_camera((0.0, 0.0, -3.0), w, h)]
        targets = _targets(rng, cams)
    elif config == 4:
        n_views = 16
        u = rng.uniform(0.0, 1.0, size=n_views)
        el = rng.uniform(-20.0, 20.0, size=n_views)
        ws = rng.integers(640, 1601, size=n_views)
        cams = []
        for k in range(n_views):
            ww = int(ws[k]) if width is None else width
            hh = int(round(0.75 * ww)) if height is None else height
            cams.append(orbit_camera(4.0, 2 * math.pi * (k + u[k]) / n_views,
                                     math.radians(el[k]), ww, hh))
        targets = _targets(rng, cams)
    else:
        n_views = 8
        u = rng.uniform(0.0, 1.0, size=n_views)
        el = rng.uniform(-20.0, 20.0, size=n_views)
        cams = []
        for k in range(n_views):
            ww = 1960 if width is None else width
            hh = 1090 if height is None else height
            cams.append(orbit_camera(4.0, 2 * math.pi * (k + u[k]) / n_views,
                                     math.radians(el[k]), ww, hh))
        targets = _targets(rng, cams)
    return Scene(params=params, sigma=10.0, background=np.zeros(3, np.float32),
                 cameras=cams, targets=targets)


def random_scene(seed, n, width, height, n_views=1, mean_range=1.0, distance=3.0,
                 log_scale_mu=-3.5, log_scale_sd=0.3, sigma=10.0):
    """Small scene for unit tests: ``n`` splats in a cube, views on an orbit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = _draw_splats(rng, n, -mean_range, mean_range, log_scale_mu, log_scale_sd)
    cams = []
    for k in range(n_views):
        if n_views == 1:
            cams.append(look_at_camera((0.0, 0.0, -distance), width, height))
        else:
            az = 2 * math.pi * (k + rng.uniform()) / n_views
            el = math.radians(rng.uniform(-20.0, 20.0))
            cams.append(orbit_camera(distance, az, el, width, height))
    targets = _targets(rng, cams)
    return Scene(params=params, sigma=sigma, background=np.zeros(3, np.float32),
                 cameras=cams, targets=targets)
