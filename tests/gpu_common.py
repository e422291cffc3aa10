"""Shared helpers of the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded inputs and compare them with the stated tolerances."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O

IMAGE_RTOL = 1e-5      # normwise: max |dC| / max |C_ref| per view
GRAD_RTOL = 1e-4       # normwise per parameter group: ||dg||_2 / ||g_ref||_2
SIGMA_RTOL = 1e-4
SIGMA_TERM_TOL = 1e-6  # of sum |terms|: dL/dsigma is a signed sum over splats that can cancel


def sigma_ok(gpu, ref, s_abs):
    """|d(dL/dsigma)| <= 1e-4 |dL/dsigma| + 1e-6 sum_i |dL/dw_i v_i d_i / sigma^2|.

    A pure relative bound is ill-posed when the terms cancel (the total can be 1e-3 of
    their magnitude on a sparse pixel sample); the second term, about 16 float32 ulps of
    the magnitude sum, is the resolution float32 inputs allow."""
    err = abs(gpu - ref)
    return err <= SIGMA_RTOL * abs(ref) + SIGMA_TERM_TOL * s_abs, err / max(abs(ref), 1e-30)
NEAR_MARGIN = 5e-5     # pairs with |255 alpha - 1| below this are float-ambiguous


def to_np(t):
    return t.detach().double().cpu().numpy()


def image_views(renderer, flat, planes=3):
    return [to_np(x) for x in renderer.views(flat, planes)]


def compare_image(gpu_img, ref, near_mask=None):
    """Normwise max error over the pixels that no near-threshold pair touches."""
    d = np.abs(gpu_img - ref)
    if near_mask is not None:
        d = d[:, ~near_mask]
        r = np.abs(ref[:, ~near_mask])
    else:
        r = np.abs(ref)
    scale = max(float(r.max()) if r.size else 0.0, 1e-30)
    return float(d.max() if d.size else 0.0) / scale


def grad_rel(g_gpu, g_ref, floor=0.0):
    """||g_gpu - g_ref||_2 / max(||g_ref||_2, floor).  ``floor`` keeps the measure
    well-posed for a group whose exact gradient vanishes (e.g. the view-weight SH of a
    splat that is alone on its pixels, where w cancels in P / Q)."""
    num = float(np.sqrt(((g_gpu - g_ref) ** 2).sum()))
    den = float(np.sqrt((g_ref ** 2).sum()))
    return num / max(den, floor, 1e-30), den


def grad_floor(g_ref: dict) -> float:
    """1e-3 of the largest group norm: float32 noise on a vanishing group must stay
    below 1e-4 of this, i.e. 1e-7 of the gradient's overall scale."""
    return 1e-3 * max(float(np.sqrt((g ** 2).sum())) for g in g_ref.values())


def oracle_grads(params, sigma, bg, cams, dLdC_views, windows=None, with_abs=False):
    """Oracle gradients summed over views.  With ``with_abs`` also returns
    sum_i |dL/dw_i v_i d_i / sigma^2|, the magnitude of the terms of dL/dsigma (its
    conditioning scale: float32 round-off on dL/dsigma is relative to this sum)."""
    tot = None
    gs = 0.0
    gabs = 0.0
    F = {f: k for k, f in enumerate(O.PROJECT_FIELDS)}
    for k, cam in enumerate(cams):
        w = windows[k] if windows else None
        g, s, scr = O.backward(params, sigma, bg, cam, dLdC_views[k], window=w, screen=with_abs)
        gs += s
        if with_abs:
            pr = O.project(params, sigma, cam)
            on = (pr[:, F["valid"]] > 0) & (pr[:, F["d"]] < sigma)
            gabs += float(np.abs(scr[:, 9] * pr[:, F["v"]] * pr[:, F["d"]] / sigma ** 2)[on].sum())
        tot = g if tot is None else {key: tot[key] + g[key] for key in tot}
    if with_abs:
        return tot, gs, gabs
    return tot, gs
