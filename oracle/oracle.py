"""Python face of the FP64 oracle.

TEST INFRASTRUCTURE: only ``tests/``, the package smoke check and the CPU-baseline leg
of the benchmark import this module.  The GPU renderer never does.

The renderer and its gradient live in ``oit_oracle.c`` (plain C, double precision,
single-threaded) and are reached here through ctypes.  The remaining, much smaller
pieces of the training step are written here in numpy float64, each as its textbook
definition:

* L1 loss and its gradient (the photometric term of the 3DGS loss, which the paper
  keeps: Sec. 5.1 "Implementation Details");
* activeness score and active-set selection (Sec. 4.1, Eq. "activeness" and the
  text after it: a splat is active if at least one attribute group's gradient norm
  exceeds its threshold; top-k selection breaks ties by the lower index);
* Adam on a subset of rows (Sec. 4.1, Alg. "Active Set Method": only the active
  splats are updated; the optimiser is Adam, Sec. 5.1);
* densification, pruning and the opacity reset of the first training phase (Sec. 5.1
  "Implementation Details": 3DGS's density control with a random keep probability),
  with the readings listed above their code.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboit_oracle.so")
SRC_PATH = os.path.join(HERE, "oit_oracle.c")

GROUPS = (("mean", 3), ("log_scale", 3), ("quat", 4), ("opacity_logit", 1), ("sh", 48), ("vsh", 16))


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               SRC_PATH, "-lm", "-o", LIB_PATH]
        subprocess.check_call(cmd)
    return LIB_PATH


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("height", ctypes.c_int),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("near_z", ctypes.c_double)]


class _Splats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_long)] + [(g, ctypes.c_void_p) for g, _ in GROUPS]


class _Grads(ctypes.Structure):
    _fields_ = [(g, ctypes.c_void_p) for g, _ in GROUPS]


class _Win(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int), ("y0", ctypes.c_int), ("x1", ctypes.c_int), ("y1", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_project.argtypes = [P, ctypes.c_double, P, P]
        L.orc_render.argtypes = [P, ctypes.c_double, P, P, P, ctypes.c_int, P, P, P, P, P,
                                 ctypes.c_double, P, P]
        L.orc_render_pixels.argtypes = [P, ctypes.c_double, P, P, ctypes.c_long, P, P, P, P, P]
        L.orc_backward.argtypes = [P, ctypes.c_double, P, P, P, P, P, P, P]
        L.orc_backward_pixels.argtypes = [P, ctypes.c_double, P, P, ctypes.c_long, P, P, P, P, P, P]
        L.orc_sh_basis.argtypes = [P, P, P]
        L.orc_quat_to_rot.argtypes = [P, P]
        for f in (L.orc_project, L.orc_render, L.orc_render_pixels, L.orc_backward,
                  L.orc_backward_pixels):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


class _Pack:
    """Holds float64 copies of the parameters and the ctypes structs pointing at them."""

    def __init__(self, params: dict):
        self.arrays = {g: np.ascontiguousarray(params[g], dtype=np.float64) for g, _ in GROUPS}
        self.n = self.arrays["mean"].shape[1]
        self.s = _Splats(self.n, *[self.arrays[g].ctypes.data for g, _ in GROUPS])


def _cam(c):
    return _Cam(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy),
                (ctypes.c_double * 9)(*np.asarray(c.R, np.float64).reshape(-1).tolist()),
                (ctypes.c_double * 3)(*np.asarray(c.t, np.float64).reshape(-1).tolist()),
                float(getattr(c, "near", 0.2)))


def _win(window, cam):
    if window is None:
        return _Win(0, 0, cam.width, cam.height)
    x0, y0, x1, y1 = window
    return _Win(int(x0), int(y0), int(x1), int(y1))


def sh_basis(direction):
    d = np.ascontiguousarray(direction, np.float64)
    Y = np.zeros(16)
    dY = np.zeros(48)
    lib().orc_sh_basis(_ptr(d), _ptr(Y), _ptr(dY))
    return Y, dY.reshape(16, 3)


def quat_to_rot(q):
    q = np.ascontiguousarray(q, np.float64)
    R = np.zeros(9)
    lib().orc_quat_to_rot(_ptr(q), _ptr(R))
    return R.reshape(3, 3)


PROJECT_FIELDS = ("valid", "mx", "my", "conic_xx", "conic_xy", "conic_yy", "opacity",
                  "c_r", "c_g", "c_b", "v", "d", "w", "tau", "cov_xx", "cov_xy", "cov_yy",
                  "x0", "x1", "y0", "y1")


def project(params, sigma, cam):
    """Per-splat screen-space quantities, [n][21] (fields in PROJECT_FIELDS)."""
    pk = _Pack(params)
    out = np.zeros((pk.n, len(PROJECT_FIELDS)))
    c = _cam(cam)
    lib().orc_project(ctypes.byref(pk.s), float(sigma), ctypes.byref(c), _ptr(out))
    return out


def render(params, sigma, bg, cam, include=None, brute=False, window=None, near_margin=0.0):
    """Dense FP64 render of one view.

    Returns dict with image [3][H][W], state [5][H][W] (T, Q, F), pre [9][H][W]
    (P0 rgb, P1 rgb, Q0, Q1, logT of the rendered subset), near [H][W] bool mask of
    pixels touched by a pair within ``near_margin`` (relative) of alpha = 1/255,
    pairs (contributing pair count) and signature (hash of all discrete decisions).
    """
    pk = _Pack(params)
    H, W = cam.height, cam.width
    image = np.zeros((3, H, W))
    state = np.zeros((5, H, W))
    pre = np.zeros((9, H, W))
    near = np.zeros((H, W), np.uint8)
    pairs = ctypes.c_longlong(0)
    sig = ctypes.c_ulonglong(0)
    inc = None if include is None else np.ascontiguousarray(include, np.uint8)
    c = _cam(cam)
    w = _win(window, cam)
    bgd = np.ascontiguousarray(bg, np.float64)
    rc = lib().orc_render(ctypes.byref(pk.s), float(sigma), _ptr(bgd), ctypes.byref(c), _ptr(inc),
                          int(bool(brute)), ctypes.byref(w), _ptr(image), _ptr(state), _ptr(pre),
                          _ptr(near), float(near_margin), ctypes.byref(pairs), ctypes.byref(sig))
    assert rc == 0
    return dict(image=image, state=state, pre=pre, near=near.astype(bool), pairs=pairs.value,
                signature=sig.value)


def render_pixels(params, sigma, bg, cam, xs, ys):
    """Pixel-major FP64 render of a list of pixels: (C [npix][3], state [npix][5], pairs)."""
    pk = _Pack(params)
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    C = np.zeros((len(xs), 3))
    st = np.zeros((len(xs), 5))
    pairs = ctypes.c_longlong(0)
    c = _cam(cam)
    bgd = np.ascontiguousarray(bg, np.float64)
    rc = lib().orc_render_pixels(ctypes.byref(pk.s), float(sigma), _ptr(bgd), ctypes.byref(c),
                                 len(xs), _ptr(xs), _ptr(ys), _ptr(C), _ptr(st), ctypes.byref(pairs))
    assert rc == 0
    return C, st, pairs.value


def _zero_grads(n):
    return {g: np.zeros((c, n)) for g, c in GROUPS}


def backward(params, sigma, bg, cam, dLdC, window=None, screen=False):
    """Gradient of sum(dLdC * C) over the window (dLdC [3][H][W]).

    Returns (grads dict [C][N] float64, d/dsigma, screen [n][10] or None).
    """
    pk = _Pack(params)
    grads = _zero_grads(pk.n)
    gr = _Grads(*[grads[g].ctypes.data for g, _ in GROUPS])
    gs = ctypes.c_double(0.0)
    scr = np.zeros((pk.n, 10)) if screen else None
    c = _cam(cam)
    w = _win(window, cam)
    g = np.ascontiguousarray(dLdC, np.float64)
    bgd = np.ascontiguousarray(bg, np.float64)
    rc = lib().orc_backward(ctypes.byref(pk.s), float(sigma), _ptr(bgd), ctypes.byref(c),
                            ctypes.byref(w), _ptr(g), ctypes.byref(gr), ctypes.byref(gs), _ptr(scr))
    assert rc == 0
    return grads, gs.value, scr


def backward_pixels(params, sigma, bg, cam, xs, ys, dLdC, screen=False):
    """Gradient of sum_k dLdC[k] . C(pixel k) for a pixel list (dLdC [npix][3]).
    Returns (grads, d/dsigma) or, with ``screen``, (grads, d/dsigma, screen [n][10])."""
    pk = _Pack(params)
    scr = np.zeros((pk.n, 10)) if screen else None
    grads = _zero_grads(pk.n)
    gr = _Grads(*[grads[g].ctypes.data for g, _ in GROUPS])
    gs = ctypes.c_double(0.0)
    xs = np.ascontiguousarray(xs, np.int32)
    ys = np.ascontiguousarray(ys, np.int32)
    g = np.ascontiguousarray(dLdC, np.float64)
    c = _cam(cam)
    bgd = np.ascontiguousarray(bg, np.float64)
    rc = lib().orc_backward_pixels(ctypes.byref(pk.s), float(sigma), _ptr(bgd), ctypes.byref(c),
                                   len(xs), _ptr(xs), _ptr(ys), _ptr(g), ctypes.byref(gr),
                                   ctypes.byref(gs), _ptr(scr))
    assert rc == 0
    if screen:
        return grads, gs.value, scr
    return grads, gs.value


# ----------------------------------------------------------------------------------
# Loss, activeness, selection and Adam (numpy float64)
# ----------------------------------------------------------------------------------

def l1_loss(image, target):
    """L = mean |C - I| over the 3HW values; dL/dC = sign(C - I) / (3HW), sign(0) = 0."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    n = d.size
    return float(np.abs(d).sum() / n), np.sign(d) / n


def activeness_score(grads: dict, rows, eps=None):
    """s_i = max over groups g of ||grad_g(i)||_2 / eps_g (Sec. 4.1, Eq. "activeness",
    read with "at least one group" as the text after it says).  ``grads`` holds the
    [C][len(rows)] gradients of the listed rows."""
    eps = eps or {g: 1.0 for g, _ in GROUPS}
    s = np.zeros(len(rows))
    for g, _ in GROUPS:
        nrm = np.sqrt((np.asarray(grads[g], np.float64) ** 2).sum(axis=0))
        s = np.maximum(s, nrm / eps[g])
    return s


def select_topk(score, k):
    """The k largest scores; ties to the lower index; returned sorted ascending."""
    score = np.asarray(score)
    order = sorted(range(len(score)), key=lambda i: (-float(score[i]), i))
    return np.array(sorted(order[:k]), dtype=np.int64)


def select_threshold(score, thresh=1.0):
    return np.nonzero(np.asarray(score) > thresh)[0].astype(np.int64)


def label_delta(old_label, new_idx, n):
    """New label byte per splat and the label changes, ascending by index.

    sign -1: the splat entered the active set (its share leaves the pre-render);
    sign +1: the splat left the active set (its share joins the pre-render).
    """
    new_label = np.zeros(n, np.uint8)
    new_label[np.asarray(new_idx, np.int64)] = 1
    old = np.asarray(old_label, np.uint8)
    changed = np.nonzero(old != new_label)[0]
    sign = np.where(new_label[changed] == 1, -1, 1).astype(np.int8)
    return new_label, changed.astype(np.int64), sign


def adam_rows(param, grad_rows, m, v, rows, lr, beta1, beta2, eps, step):
    """Adam on the listed rows of a [C][N] parameter (in place, float64).

    grad_rows is [C][len(rows)] in the order of ``rows``.  Bias correction uses the
    global step count; rows not listed keep their values and moments untouched.
    """
    rows = np.asarray(rows, np.int64)
    g = np.asarray(grad_rows, np.float64)
    m[:, rows] = beta1 * m[:, rows] + (1.0 - beta1) * g
    v[:, rows] = beta2 * v[:, rows] + (1.0 - beta2) * g * g
    mhat = m[:, rows] / (1.0 - beta1 ** step)
    vhat = v[:, rows] / (1.0 - beta2 ** step)
    param[:, rows] = param[:, rows] - lr * mhat / (np.sqrt(vhat) + eps)


def fps(centres, s, start):
    """Farthest-point sampling over camera centres (Sec. 4.1: the active set is updated
    on a subset of training views chosen by farthest point sampling from a random
    start).  Picks ``start``, then repeatedly the point whose squared distance to the
    nearest picked point is largest (first such index on ties)."""
    c = np.asarray(centres, dtype=np.float32).astype(np.float64)
    picked = [int(start)]
    d = ((c - c[start]) ** 2).sum(axis=1)
    for _ in range(int(s) - 1):
        j = int(np.argmax(d))
        picked.append(j)
        d = np.minimum(d, ((c - c[j]) ** 2).sum(axis=1))
    return picked


# ----------------------------------------------------------------------------------
# D-SSIM: the structural term of the 3DGS loss that the paper keeps (Sec. 5.1,
# "Implementation Details": the loss and lambda_ssim follow 3DGS).  Reading: SSIM with an
# 11 x 11 Gaussian window (std 1.5, normalised), zero padding ("same" size), constants
# C1 = 0.01^2, C2 = 0.03^2, averaged over the 3HW values; D-SSIM = 1 - SSIM and the
# loss (1 - lambda) L1 + lambda D-SSIM with lambda = 0.2, summed over views.
# ----------------------------------------------------------------------------------
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2


def gaussian_window(size=11, std=1.5):
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-x * x / (2.0 * std * std))
    return g / g.sum()


def _filter(img, g):
    """Zero-padded 'same' 2D filtering of [H][W] with the separable window g (rows, then
    columns), written as explicit shifted sums."""
    H, W = img.shape
    r = len(g) // 2
    tmp = np.zeros_like(img)
    for k, gk in enumerate(g):
        d = k - r
        if d >= 0:
            tmp[:, :W - d] += gk * img[:, d:]
        else:
            tmp[:, -d:] += gk * img[:, :W + d]
    out = np.zeros_like(img)
    for k, gk in enumerate(g):
        d = k - r
        if d >= 0:
            out[:H - d, :] += gk * tmp[d:, :]
        else:
            out[-d:, :] += gk * tmp[:H + d, :]
    return out


def ssim_map(x, y):
    """Per-pixel SSIM of two [3][H][W] images (float64)."""
    g = gaussian_window()
    S = np.zeros_like(np.asarray(x, np.float64))
    for ch in range(3):
        a = np.asarray(x[ch], np.float64)
        b = np.asarray(y[ch], np.float64)
        mx, my = _filter(a, g), _filter(b, g)
        sxx = _filter(a * a, g) - mx * mx
        syy = _filter(b * b, g) - my * my
        sxy = _filter(a * b, g) - mx * my
        S[ch] = ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / \
                ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))
    return S


def dssim_loss_grad(x, y):
    """D-SSIM = 1 - mean(SSIM) of image x against target y and its gradient wrt x.

    With S = A1 A2 / (B1 B2), A1 = 2 mx my + C1, A2 = 2 (Exy - mx my) + C2,
    B1 = mx^2 + my^2 + C1, B2 = Exx - mx^2 + Eyy - my^2 + C2 (E = filtered products):
      dS/dmx = S (2my/A1 - 2my/A2 - 2mx/B1 + 2mx/B2),  dS/dExx = -S/B2,  dS/dExy = 2S/A2,
    and dmean(S)/dx = [g * dS/dmx + 2x (g * dS/dExx) + y (g * dS/dExy)] / (3HW), the
    filtering being its own adjoint for the symmetric window with zero padding."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    g = gaussian_window()
    M = x.size
    grad = np.zeros_like(x)
    total = 0.0
    for ch in range(3):
        a, b = x[ch], y[ch]
        mx, my = _filter(a, g), _filter(b, g)
        Exx, Eyy, Exy = _filter(a * a, g), _filter(b * b, g), _filter(a * b, g)
        A1 = 2 * mx * my + SSIM_C1
        A2 = 2 * (Exy - mx * my) + SSIM_C2
        B1 = mx * mx + my * my + SSIM_C1
        B2 = (Exx - mx * mx) + (Eyy - my * my) + SSIM_C2
        S = A1 * A2 / (B1 * B2)
        total += S.sum()
        dmx = S * (2 * my / A1 - 2 * my / A2 - 2 * mx / B1 + 2 * mx / B2)
        dExx = -S / B2
        dExy = 2 * S / A2
        grad[ch] = -(_filter(dmx, g) + 2 * a * _filter(dExx, g) + b * _filter(dExy, g)) / M
    return 1.0 - total / M, grad


def l1_dssim_loss(image, target, lam=0.2):
    """(1 - lambda) L1 + lambda D-SSIM of one view, and its gradient."""
    l1, g1 = l1_loss(image, target)
    ds, g2 = dssim_loss_grad(image, target)
    return (1 - lam) * l1 + lam * ds, (1 - lam) * g1 + lam * g2


# ----------------------------------------------------------------------------------
# Densification and pruning (numpy float64).  The paper trains its first phase as
# 3DGS does, densification included, and keeps 3DGS's density control, adding a
# scene-specific random keep probability that caps the splat count (Sec. 5.1
# "Implementation Details"; Fig. "overview": the active-set phase starts after it).
# The rules themselves are those of 3DGS's adaptive density control, which the paper
# adopts without restating; the readings are:
#   * statistic: per (splat, view) where the splat is visible, the norm of the loss
#     gradient with respect to its projected mean expressed per normalised-device
#     unit (pixel gradient times W / 2 and H / 2), summed over views, with the
#     number of visible views and the largest 3-sigma screen radius;
#   * visible: the projection is valid, opacity >= 1/255, and the footprint box of
#     the alpha >= 1/255 ellipse contains at least one pixel centre of the image;
#   * a splat is a candidate when its mean statistic reaches the threshold and its
#     uniform draw is below the keep probability (these comparisons, which decide what
#     exists, in float32: the kernels' precision); a small candidate (largest scale
#     <= percent_dense * extent) is cloned, a large one is replaced by two children
#     drawn from its Gaussian (mean + R diag(s) z) with scales divided by 1.6;
#   * pruning applies to the densified set: every splat below the minimum opacity,
#     every splat whose largest scale exceeds max_world_frac * extent, and every
#     original splat whose recorded screen radius exceeds max_screen_size;
#   * order of the new set: surviving originals, then clone copies, then the first
#     children of the split splats, then their second children, each in source order;
#     new splats start with zero Adam moments.
# ----------------------------------------------------------------------------------
from dataclasses import dataclass  # noqa: E402

SPLIT_DIVISOR = 1.6


@dataclass
class DensityRules:
    grad_threshold: float = 0.0002
    percent_dense: float = 0.01
    scene_extent: float = 1.0
    min_opacity: float = 0.005
    max_screen_size: float = 0.0    # <= 0: off
    max_world_frac: float = 0.0     # <= 0: off
    keep_probability: float = 1.0


def footprint_visible(pr_row, width, height):
    """Whether a projected splat (a row of project()) reaches a pixel centre of the image."""
    valid, mx, my, tau = pr_row[0], pr_row[1], pr_row[2], pr_row[13]
    if not valid or tau < 0.0:
        return False
    hx, hy = math.sqrt(tau * pr_row[14]), math.sqrt(tau * pr_row[16])
    x_lo, x_hi = math.ceil(mx - hx - 0.5), math.floor(mx + hx - 0.5)
    y_lo, y_hi = math.ceil(my - hy - 0.5), math.floor(my + hy - 0.5)
    return max(x_lo, 0) <= min(x_hi, width - 1) and max(y_lo, 0) <= min(y_hi, height - 1)


def screen_radius(pr_row):
    """3 sigma of the major axis of the screen covariance (pixels)."""
    a, b, c = pr_row[14], pr_row[15], pr_row[16]
    lam = 0.5 * (a + c) + math.sqrt(0.25 * (a - c) ** 2 + b * b)
    return 3.0 * math.sqrt(lam)


def densify_stats(params, sigma, bg, cams, dLdCs, accum=None, denom=None, max_radius=None):
    """Accumulate the densification statistic over the views (dLdCs[k] [3][H][W])."""
    n = params["mean"].shape[1]
    accum = np.zeros(n) if accum is None else accum
    denom = np.zeros(n) if denom is None else denom
    max_radius = np.zeros(n) if max_radius is None else max_radius
    for cam, g in zip(cams, dLdCs):
        pr = project(params, sigma, cam)
        _, _, scr = backward(params, sigma, bg, cam, g, screen=True)
        for i in range(n):
            if not footprint_visible(pr[i], cam.width, cam.height):
                continue
            accum[i] += math.hypot(scr[i, 0] * cam.width / 2.0, scr[i, 1] * cam.height / 2.0)
            denom[i] += 1.0
            max_radius[i] = max(max_radius[i], screen_radius(pr[i]))
    return accum, denom, max_radius


def densify_decisions(params, accum, denom, max_radius, uniform, rules: DensityRules):
    """Per splat: (clone, split, keep_original, keep_clone, keep_children) boolean arrays,
    every comparison in float64 (the paper fixes no precision for them)."""
    f = np.float64
    accum, denom = np.asarray(accum, f), np.asarray(denom, f)
    avg = np.where(denom > 0, accum / np.where(denom > 0, denom, f(1)), f(0))
    cand = (avg >= f(rules.grad_threshold)) & (np.asarray(uniform, f) < f(rules.keep_probability))
    smax = np.exp(np.asarray(params["log_scale"], f)).max(axis=0)
    small = smax <= f(rules.percent_dense) * f(rules.scene_extent)
    clone, split = cand & small, cand & ~small
    low = f(1) / (f(1) + np.exp(-np.asarray(params["opacity_logit"][0], f))) < f(rules.min_opacity)

    def world_big(s):
        if rules.max_world_frac <= 0:
            return np.zeros(s.shape, bool)
        return s > f(rules.max_world_frac) * f(rules.scene_extent)

    screen_big = (np.asarray(max_radius, f) > f(rules.max_screen_size)) if rules.max_screen_size > 0 \
        else np.zeros(len(smax), bool)
    keep_orig = ~split & ~low & ~screen_big & ~world_big(smax)
    keep_clone = clone & ~low & ~world_big(smax)
    keep_children = split & ~low & ~world_big(smax / f(SPLIT_DIVISOR))
    return clone, split, keep_orig, keep_clone, keep_children


def split_child(params, i, z):
    """Parameters of a child of splat i for the standard normal draw z [3]."""
    q = params["quat"][:, i] / np.linalg.norm(params["quat"][:, i])
    R = quat_to_rot(q)
    s = np.exp(params["log_scale"][:, i])
    child = {g: params[g][:, i].copy() for g, _ in GROUPS}
    child["mean"] = params["mean"][:, i] + R @ (s * np.asarray(z, np.float64))
    child["log_scale"] = params["log_scale"][:, i] - math.log(SPLIT_DIVISOR)
    return child


def densify(params, m, v, accum, denom, max_radius, uniform, normals, rules: DensityRules):
    """The densified and pruned set: (params, m, v, source) with source[j] the splat
    that new splat j comes from.  normals [n][2][3]: the draws of the two children."""
    clone, split, keep_orig, keep_clone, keep_children = densify_decisions(
        params, accum, denom, max_radius, uniform, rules)
    cols, src, fresh = [], [], []
    for i in np.flatnonzero(keep_orig):
        cols.append({g: params[g][:, i] for g, _ in GROUPS}); src.append(i); fresh.append(False)
    for i in np.flatnonzero(keep_clone):
        cols.append({g: params[g][:, i] for g, _ in GROUPS}); src.append(i); fresh.append(True)
    for k in range(2):
        for i in np.flatnonzero(keep_children):
            cols.append(split_child(params, i, normals[i][k])); src.append(i); fresh.append(True)
    n_new = len(cols)
    out_p = {g: np.zeros((c, n_new)) for g, c in GROUPS}
    out_m = {g: np.zeros((c, n_new)) for g, c in GROUPS}
    out_v = {g: np.zeros((c, n_new)) for g, c in GROUPS}
    for j, col in enumerate(cols):
        for g, _ in GROUPS:
            out_p[g][:, j] = col[g]
            if not fresh[j]:
                out_m[g][:, j] = m[g][:, src[j]]
                out_v[g][:, j] = v[g][:, src[j]]
    return out_p, out_m, out_v, np.asarray(src, np.int64)


def reset_opacity(params, m, v, max_opacity=0.01):
    """Opacity reset of 3DGS: every opacity is clamped to max_opacity and the opacity
    group's Adam moments restart from zero."""
    cap = math.log(max_opacity / (1.0 - max_opacity))
    params["opacity_logit"] = np.minimum(params["opacity_logit"], cap)
    m["opacity_logit"] = np.zeros_like(m["opacity_logit"])
    v["opacity_logit"] = np.zeros_like(v["opacity_logit"])
    return params, m, v
