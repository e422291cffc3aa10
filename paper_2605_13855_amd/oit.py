"""ctypes binding of liboit (argument marshalling only).

Each function here has the name of the C entry point without its ``oit_`` prefix,
takes torch tensors (device memory) or ``None``, and passes their data pointers and
the current HIP stream of torch to the library.  Every computation happens in the
library's HIP kernels; nothing here computes on the host.  The module raises at
import if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboit.so")

OK = 0
STATUS_PAIR_OVERFLOW = 1
STATUS_ACTIVE_OVERFLOW = 2
STATUS_DELTA_OVERFLOW = 4
SELECT_TOPK = 0
SELECT_THRESHOLD = 1
MAX_VIEWS = 64
PIXSTATE_PLANES = 6   # T, Q, F (rgb), dQ/dsigma (OIT_PIXSTATE_PLANES)
GROUPS = (("mean", 3), ("log_scale", 3), ("quat", 4), ("opacity_logit", 1), ("sh", 48), ("vsh", 16))


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3),
                ("near_z", ctypes.c_float)]


class Splats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64)] + [(g, ctypes.c_void_p) for g, _ in GROUPS]


class Grads(ctypes.Structure):
    _fields_ = [(g, ctypes.c_void_p) for g, _ in GROUPS] + [("stride", ctypes.c_int64)]


BWD_PER_SPLAT = 0
BWD_PER_PIXEL = 1


class Tuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("batch", ctypes.c_int32), ("pair_capacity", ctypes.c_int64),
                ("bwd_mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Capacity(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("active_capacity", ctypes.c_int64),
                ("delta_capacity", ctypes.c_int64)]


class OITError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise OITError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, F, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
    L.oit_workspace_bytes.argtypes = [P, P, I32, P]
    L.oit_workspace_bytes.restype = SZ
    L.oit_render_fwd.argtypes = [P, P, P, P, I32, P, P, P, P, P, P, P, P, P, P, P, SZ, P, P]
    L.oit_l1_loss.argtypes = [P, P, P, I32, P, P, P, SZ, P]
    L.oit_l1_loss_workspace_bytes.argtypes = []
    L.oit_l1_loss_workspace_bytes.restype = SZ
    L.oit_render_bwd.argtypes = [P, P, P, P, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, P, SZ, P, P]
    L.oit_select_workspace_bytes.argtypes = [I64]
    L.oit_select_workspace_bytes.restype = SZ
    L.oit_update_active_set.argtypes = [P, I64, I32, I64, F, P, P, I64, P, P, P, I64, P, P, SZ, P]
    L.oit_update_active_set_noalloc.argtypes = [P, I64, I32, I64, F, P, P, I64, P, P, P, I64, P, P, P]
    L.oit_sparse_adam_step.argtypes = [P, P, P, P, P, P, I64, P, F, F, F, P, P]
    L.oit_sigma_adam_step.argtypes = [P, P, P, P, F, F, F, F, P, P]
    L.oit_read_status.argtypes = [P, SZ, P, P]
    L.oit_clear_status.argtypes = [P, SZ, P]
    L.oit_read_counters.argtypes = [P, SZ, P, P, I32, P, P, P]
    L.oit_loss_workspace_bytes.argtypes = [P, I32]
    L.oit_loss_workspace_bytes.restype = SZ
    L.oit_l1_dssim_loss.argtypes = [P, P, P, I32, F, P, P, P, SZ, P]
    L.oit_l1_dssim_loss.restype = ctypes.c_int
    L.oit_label_delta.argtypes = [P, P, I64, P, I64, P, P, P, I64, P, P, SZ, P]
    L.oit_fps_views.argtypes = [P, I32, I32, I32, P]
    L.oit_densify_stats.argtypes = [P, I32, P, P, P, P, P, P, P, P, SZ, P, P]
    L.oit_densify_workspace_bytes.argtypes = [I64]
    L.oit_densify_workspace_bytes.restype = SZ
    L.oit_densify_plan.argtypes = [P, P, P, P, P, P, P, P, SZ, P]
    L.oit_densify_apply.argtypes = [P, P, P, P, P, P, P, I64, P, SZ, P]
    L.oit_reset_opacity.argtypes = [P, P, P, I64, F, P]
    L.oit_timing_enable.argtypes = [I32]
    L.oit_timing_read.argtypes = [P]
    L.oit_read_tile_entries.argtypes = [P, SZ, P, P, I32, P, P, I64, P]
    L.oit_timing_read_stages.argtypes = [P]
    L.oit_last_error.argtypes = []
    L.oit_last_error.restype = ctypes.c_char_p
    for f in (L.oit_render_fwd, L.oit_l1_loss, L.oit_render_bwd, L.oit_update_active_set,
              L.oit_update_active_set_noalloc,
              L.oit_sparse_adam_step, L.oit_sigma_adam_step, L.oit_read_status, L.oit_clear_status,
              L.oit_read_counters, L.oit_read_tile_entries, L.oit_timing_enable, L.oit_timing_read,
              L.oit_timing_read_stages,
              L.oit_label_delta,
              L.oit_fps_views, L.oit_densify_stats, L.oit_densify_plan, L.oit_densify_apply,
              L.oit_reset_opacity):
        f.restype = ctypes.c_int
    return L


lib = _load()


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    if not t.is_contiguous():
        raise OITError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, what):
    if rc != OK:
        raise OITError(f"{what} failed ({rc}): {lib.oit_last_error().decode()}")


def camera_struct(cam) -> Camera:
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = [float(x) for x in list(getattr(cam.R, "reshape")(-1))]
    t = [float(x) for x in list(getattr(cam.t, "reshape")(-1))]
    c.R = (ctypes.c_float * 9)(*R)
    c.t = (ctypes.c_float * 3)(*t)
    c.near_z = float(getattr(cam, "near", 0.2))
    return c


def camera_array(cams):
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


def splats_struct(params: dict) -> Splats:
    n = params["mean"].shape[0]
    for g, c in GROUPS:
        t = params[g]
        if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != (n, c):
            raise OITError(f"parameter {g} must be contiguous float32 [{n}][{c}] (splat-major)")
    return Splats(n, *[params[g].data_ptr() for g, _ in GROUPS])


def grads_struct(grads: dict, stride: int) -> Grads:
    return Grads(*[grads[g].data_ptr() for g, _ in GROUPS], int(stride))


def workspace_bytes(cap: Capacity, cams_arr, n_views: int, tuning: Tuning) -> int:
    return int(lib.oit_workspace_bytes(ctypes.byref(cap), cams_arr, n_views, ctypes.byref(tuning)))


def render_fwd(splats: Splats, sigma, bg_host, cams_arr, n_views, cap: Capacity, active_idx, n_active,
               delta_idx, delta_sign, n_delta, pre, image, pixstate, ws, tuning: Tuning, stream=None,
               delta_splats: Splats = None):
    bg = (ctypes.c_float * 3)(*[float(x) for x in bg_host])
    rc = lib.oit_render_fwd(ctypes.byref(splats), _ptr(sigma), bg, cams_arr, n_views, ctypes.byref(cap),
                            _ptr(active_idx), _ptr(n_active), _ptr(delta_idx), _ptr(delta_sign), _ptr(n_delta),
                            ctypes.byref(delta_splats) if delta_splats is not None else None,
                            _ptr(pre), _ptr(image), _ptr(pixstate), _ptr(ws), ws.numel(),
                            ctypes.byref(tuning), _stream(stream))
    _check(rc, "oit_render_fwd")


def l1_loss(image, target, cams_arr, n_views, grad_image, loss, ws, stream=None):
    rc = lib.oit_l1_loss(_ptr(image), _ptr(target), cams_arr, n_views, _ptr(grad_image), _ptr(loss),
                         _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "oit_l1_loss")


def l1_loss_workspace_bytes() -> int:
    return int(lib.oit_l1_loss_workspace_bytes())


def loss_workspace_bytes(cams_arr, n_views) -> int:
    return int(lib.oit_loss_workspace_bytes(cams_arr, int(n_views)))


def l1_dssim_loss(image, target, cams_arr, n_views, lam, grad_image, loss, ws, stream=None):
    rc = lib.oit_l1_dssim_loss(_ptr(image), _ptr(target), cams_arr, int(n_views), float(lam), _ptr(grad_image),
                               _ptr(loss), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "oit_l1_dssim_loss")


def render_bwd(splats: Splats, sigma, bg_host, cams_arr, n_views, cap: Capacity, active_idx, n_active,
               delta_idx, delta_sign, n_delta, pre, grad_image, pixstate, grads: Grads, grad_sigma, score,
               eps_host, ws, tuning: Tuning, stream=None):
    bg = (ctypes.c_float * 3)(*[float(x) for x in bg_host])
    eps = None if eps_host is None else (ctypes.c_float * 6)(*[float(x) for x in eps_host])
    rc = lib.oit_render_bwd(ctypes.byref(splats), _ptr(sigma), bg, cams_arr, n_views, ctypes.byref(cap),
                            _ptr(active_idx), _ptr(n_active), _ptr(delta_idx), _ptr(delta_sign), _ptr(n_delta),
                            _ptr(pre), _ptr(grad_image), _ptr(pixstate), ctypes.byref(grads), _ptr(grad_sigma),
                            _ptr(score), eps, _ptr(ws), ws.numel(), ctypes.byref(tuning), _stream(stream))
    _check(rc, "oit_render_bwd")


def select_workspace_bytes(n: int) -> int:
    return int(lib.oit_select_workspace_bytes(int(n)))


def update_active_set(score, n, mode, k, thresh, label, active_idx, n_active, delta_idx, delta_sign, n_delta,
                      ws, stream=None):
    rc = lib.oit_update_active_set(_ptr(score), int(n), int(mode), int(k), float(thresh), _ptr(label),
                                   _ptr(active_idx), active_idx.numel(), _ptr(n_active), _ptr(delta_idx),
                                   _ptr(delta_sign), delta_idx.numel(), _ptr(n_delta), _ptr(ws), ws.numel(),
                                   _stream(stream))
    _check(rc, "oit_update_active_set")


NOALLOC_SELECT_MAX_N = 1 << 22   # OIT_NOALLOC_SELECT_MAX_N


def update_active_set_noalloc(score, n, mode, k, thresh, label, active_idx, n_active, delta_idx, delta_sign,
                              n_delta, status, stream=None):
    """update_active_set without a workspace (the library's static per-GPU scratch);
    status: [1] device int32 output of the overflow bits."""
    rc = lib.oit_update_active_set_noalloc(_ptr(score), int(n), int(mode), int(k), float(thresh), _ptr(label),
                                           _ptr(active_idx), active_idx.numel(), _ptr(n_active), _ptr(delta_idx),
                                           _ptr(delta_sign), delta_idx.numel(), _ptr(n_delta), _ptr(status),
                                           _stream(stream))
    _check(rc, "oit_update_active_set_noalloc")


def label_delta(old_label, new_label, n, active_idx, n_active, delta_idx, delta_sign, n_delta, ws, stream=None):
    rc = lib.oit_label_delta(_ptr(old_label), _ptr(new_label), int(n), _ptr(active_idx),
                             active_idx.numel() if active_idx is not None else 0, _ptr(n_active), _ptr(delta_idx),
                             delta_sign.data_ptr() if delta_sign is not None else None, delta_idx.numel(),
                             _ptr(n_delta), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "oit_label_delta")


def fps_views(centres, s: int, start: int):
    """centres: host float array [n][3]; returns the s picked view indices."""
    import numpy as np
    c = np.ascontiguousarray(centres, dtype=np.float32)
    out = (ctypes.c_int32 * int(s))()
    rc = lib.oit_fps_views(ctypes.c_void_p(c.ctypes.data), int(c.shape[0]), int(s), int(start), out)
    _check(rc, "oit_fps_views")
    return [int(x) for x in out]


def sparse_adam_step(params: dict, grads: Grads, m: dict, v: dict, active_idx, n_active, n, lr, beta1, beta2,
                     eps, step, stream=None):
    P6 = ctypes.c_void_p * 6
    for g, c in GROUPS:
        for name, d in (("params", params), ("m", m), ("v", v)):
            t = d[g]
            if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != (int(n), c):
                raise OITError(f"{name}[{g}] must be contiguous float32 [{int(n)}][{c}] (splat-major)")
    pp = P6(*[params[g].data_ptr() for g, _ in GROUPS])
    mm = P6(*[m[g].data_ptr() for g, _ in GROUPS])
    vv = P6(*[v[g].data_ptr() for g, _ in GROUPS])
    lrs = (ctypes.c_float * 6)(*[float(x) for x in lr])
    rc = lib.oit_sparse_adam_step(pp, ctypes.byref(grads), mm, vv, _ptr(active_idx), _ptr(n_active), int(n), lrs,
                                  float(beta1), float(beta2), float(eps), _ptr(step), _stream(stream))
    _check(rc, "oit_sparse_adam_step")


def sigma_adam_step(sigma, grad_sigma, m, v, lr, beta1, beta2, eps, step, stream=None):
    rc = lib.oit_sigma_adam_step(_ptr(sigma), _ptr(grad_sigma), _ptr(m), _ptr(v), float(lr), float(beta1),
                                 float(beta2), float(eps), _ptr(step), _stream(stream))
    _check(rc, "oit_sigma_adam_step")


def read_status(ws, stream=None) -> int:
    out = ctypes.c_int32(0)
    rc = lib.oit_read_status(_ptr(ws), ws.numel(), ctypes.byref(out), _stream(stream))
    _check(rc, "oit_read_status")
    return int(out.value)


def read_counters(ws, cap: Capacity, cams_arr, n_views, tuning: Tuning, stream=None):
    """(entries needed, contributing pairs, evaluated pairs, backward work items, items the
    backward walked box by box, items it walked group by group with the whole wave) of the
    last forward / backward on this workspace."""
    out = (ctypes.c_int64 * 6)()
    rc = lib.oit_read_counters(_ptr(ws), ws.numel(), ctypes.byref(cap), cams_arr, n_views, ctypes.byref(tuning),
                               out, _stream(stream))
    _check(rc, "oit_read_counters")
    return tuple(int(x) for x in out)


def read_tile_entries(ws, cap: Capacity, cams_arr, n_views, tuning: Tuning, n_tiles: int, stream=None):
    """Per-tile (active, label-change) entry counts of the last forward: numpy [2][T]."""
    import numpy as np
    out = np.zeros(2 * n_tiles, dtype=np.uint32)
    rc = lib.oit_read_tile_entries(_ptr(ws), ws.numel(), ctypes.byref(cap), cams_arr, n_views,
                                   ctypes.byref(tuning), out.ctypes.data_as(ctypes.c_void_p), out.size,
                                   _stream(stream))
    _check(rc, "oit_read_tile_entries")
    return out.reshape(2, n_tiles)


def timing_enable(on: bool):
    _check(lib.oit_timing_enable(1 if on else 0), "oit_timing_enable")


def timing_read():
    out = (ctypes.c_float * 2)()
    _check(lib.oit_timing_read(out), "oit_timing_read")
    return float(out[0]), float(out[1])


STAGES = ("preprocess", "binning", "raster_fwd", "pixconst", "raster_bwd", "preprocess_bwd")


def timing_read_stages():
    """Milliseconds of the last render_fwd's and render_bwd's stages (STAGES order)."""
    out = (ctypes.c_float * 6)()
    _check(lib.oit_timing_read_stages(out), "oit_timing_read_stages")
    return dict(zip(STAGES, (float(x) for x in out)))


def clear_status(ws, stream=None):
    rc = lib.oit_clear_status(_ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "oit_clear_status")


# ----------------------------------------------------------------------------------
# densification of the first training phase
# ----------------------------------------------------------------------------------
class DensityRules(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("percent_dense", ctypes.c_float),
                ("scene_extent", ctypes.c_float), ("min_opacity", ctypes.c_float),
                ("max_screen_size", ctypes.c_float), ("max_world_frac", ctypes.c_float),
                ("keep_probability", ctypes.c_float), ("reserved", ctypes.c_int32)]


def densify_stats(cams_arr, n_views, cap: Capacity, active_idx, n_active, n_delta, grad_accum, denom, max_radius,
                  ws, tuning: Tuning, stream=None):
    rc = lib.oit_densify_stats(cams_arr, n_views, ctypes.byref(cap), _ptr(active_idx), _ptr(n_active),
                               _ptr(n_delta), _ptr(grad_accum), _ptr(denom), _ptr(max_radius), _ptr(ws),
                               ws.numel(), ctypes.byref(tuning), _stream(stream))
    _check(rc, "oit_densify_stats")


def densify_workspace_bytes(n: int) -> int:
    return int(lib.oit_densify_workspace_bytes(int(n)))


def densify_plan(splats: Splats, grad_accum, denom, max_radius, uniform, rules: DensityRules, n_new, ws,
                 stream=None):
    rc = lib.oit_densify_plan(ctypes.byref(splats), _ptr(grad_accum), _ptr(denom), _ptr(max_radius),
                              _ptr(uniform), ctypes.byref(rules), _ptr(n_new), _ptr(ws), ws.numel(),
                              _stream(stream))
    _check(rc, "oit_densify_plan")


def densify_apply(splats: Splats, m: dict, v: dict, normals, params_new: dict, m_new: dict, v_new: dict,
                  cap_new: int, ws, stream=None):
    P6 = ctypes.c_void_p * 6
    arr = lambda d: P6(*[d[g].data_ptr() for g, _ in GROUPS])
    rc = lib.oit_densify_apply(ctypes.byref(splats), arr(m), arr(v), _ptr(normals), arr(params_new), arr(m_new),
                               arr(v_new), int(cap_new), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "oit_densify_apply")


def reset_opacity(opacity_logit, m_opacity, v_opacity, n, max_opacity, stream=None):
    rc = lib.oit_reset_opacity(_ptr(opacity_logit), _ptr(m_opacity), _ptr(v_opacity), int(n), float(max_opacity),
                               _stream(stream))
    _check(rc, "oit_reset_opacity")
