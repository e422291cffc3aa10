"""Shared helpers of the GPU parity tests: run the HIP path and the FP64 oracle on the
same seeded inputs and compare them with the stated tolerances."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O

IMAGE_RTOL = 1e-5      # normwise: max |dC| / max |C_ref| per view
GRAD_RTOL = 1e-4       # normwise per parameter group: ||dg||_2 / ||g_ref||_2
SIGMA_RTOL = 1e-4
SIGMA_FLOOR = 1e-3     # of sum |terms|, where the exact dL/dsigma vanishes
# per row of a group: ||dg_row|| / max(||g_row||, 1e-3 largest row norm).  float32
# rounding of a row whose own terms cancel reaches ~1e-3 at that floor (measured worst
# 1.1e-3, the opacity row of a sub-pixel splat); a fault in one splat's gradient (a
# dropped tile entry, a wrong partial or index) is an O(1) error there
ROW_RTOL = 1e-2


def sigma_ok(gpu, ref, s_abs):
    """|d(dL/dsigma)| <= 1e-4 max(|dL/dsigma|, 1e-3 sum_i |dL/dw_i dw_i/dsigma|).

    The bound is relative; the floor keeps it well-posed where the exact value vanishes
    (a splat alone on its pixels has F = c, so dL/dw = 0) and takes effect only when the
    terms cancel to below a thousandth of their magnitude.  Returns (ok, relative error)."""
    err = abs(gpu - ref)
    return err <= SIGMA_RTOL * max(abs(ref), SIGMA_FLOOR * s_abs), err / max(abs(ref), 1e-30)


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


def row_rel(g_gpu, g_ref, floor=0.0):
    """Largest per-row error of one group [C][rows]: ||dg[:, r]||_2 / max(||g_ref[:, r]||_2,
    1e-3 max_r ||g_ref[:, r]||_2, floor).  A single wrong splat among thousands, which
    the group norm hides, shows here.  ``floor`` (the group check's) keeps a group whose
    exact gradient vanishes well-posed."""
    if g_ref.shape[1] == 0:
        return 0.0
    num = np.sqrt(((g_gpu - g_ref) ** 2).sum(0))
    den = np.sqrt((g_ref ** 2).sum(0))
    floor = max(1e-3 * float(den.max()), floor, 1e-30)
    return float((num / np.maximum(den, floor)).max())


def compare_grads(g_gpu: dict, g_ref: dict, log, tag=""):
    """Every group normwise within GRAD_RTOL and every row within ROW_RTOL.
    g_gpu, g_ref: {group: [C][rows] float64}."""
    fl = grad_floor(g_ref)
    worst = (0.0, 0.0)
    for name, _ in O.GROUPS:
        rel, den = grad_rel(g_gpu[name], g_ref[name], fl)
        rr = row_rel(g_gpu[name], g_ref[name], fl)
        log(f"  {tag}grad {name}: rel {rel:.2e} (norm {den:.3e}), worst row {rr:.2e}")
        assert rel <= GRAD_RTOL, (tag, name, rel)
        assert rr <= ROW_RTOL, (tag, name, rr)
        worst = (max(worst[0], rel), max(worst[1], rr))
    return worst


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
