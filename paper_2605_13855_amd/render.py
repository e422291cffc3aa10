"""Renderer, autograd function and active-set training iteration on top of liboit.

Everything that computes is a liboit call (see ``oit.py``); this module owns the
device buffers (through torch) and sequences the calls:

* ``Renderer``: cameras, capacities, tuning and the workspace of one batch of views;
  ``forward`` / ``backward`` are the two passes of the OIT rasteriser.
* ``OITRender``: a ``torch.autograd.Function`` over the dense renderer; its
  backward reuses the forward's tile lists and per-pixel totals (T, Q, F) and
  recomputes the per-pair weights instead of storing per-pixel splat lists.
* ``ActiveSetTrainer``: one iteration of Alg. "Active Set Method" (Sec. 4.1) on a
  batch of views: select the active set from the last scores, render the active
  splats against the pre-rendered inactive set (updating it with the label
  changes), L1 loss, backward on the active rows, sparse Adam, Adam on sigma.  The
  whole iteration can be captured once into a HIP graph and replayed.
"""
from __future__ import annotations

import math

import torch

from . import oit

GROUPS = oit.GROUPS


def params_to_device(params: dict, device="cuda") -> dict:
    """Component-major host arrays ([C][n], the scene generator's layout) to the
    splat-major device tensors the library takes ([n][C])."""
    return {g: torch.as_tensor(params[g], dtype=torch.float32).t().contiguous().to(device) for g, _ in GROUPS}


def params_to_host(params: dict) -> dict:
    """Splat-major device tensors back to component-major float32 host arrays."""
    return {g: params[g].detach().t().contiguous().cpu().numpy() for g, _ in GROUPS}


def _aligned_workspace(nbytes: int, device) -> torch.Tensor:
    buf = torch.zeros(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def estimate_pairs(n_listed: int, cams, tile: int, log_scale_mu=-3.5, depth=3.0) -> int:
    """Rough (tile, splat) entry estimate used to size the first pair capacity (the
    forward reports the exact need, see Renderer.fit_pair_capacity)."""
    tot = 0.0
    for c in cams:
        f = float(c.fx)
        r = 3.3 * f * math.exp(log_scale_mu) / depth + 1.0       # footprint radius, px
        tiles = (2 * r / tile + 1.5) ** 2
        tot += n_listed * min(tiles, (c.width / tile + 1) * (c.height / tile + 1))
    return int(tot * 1.5) + 4096


class Renderer:
    """One batch of views: workspace, per-pixel buffers and the two passes."""

    def __init__(self, cams, n, active_capacity=None, delta_capacity=0, tile=16, batch=64,
                 pair_capacity=None, device="cuda"):
        self.device = torch.device(device)
        self.cams = list(cams)
        self.n_views = len(self.cams)
        self.cams_arr = oit.camera_array(self.cams)
        self.n = int(n)
        self.cap = oit.Capacity(self.n, int(active_capacity or self.n), int(delta_capacity))
        self.hw = [c.height * c.width for c in self.cams]
        self.total_px = sum(self.hw)
        if pair_capacity is None:
            pair_capacity = min(estimate_pairs(self.cap.active_capacity + self.cap.delta_capacity,
                                               self.cams, tile), 2 ** 32 - 2)
        self.tuning = oit.Tuning(int(tile), int(batch), int(pair_capacity), oit.BWD_PER_SPLAT, 0)
        self._alloc_ws()
        dev = self.device
        self._image_buf = torch.zeros(3 * self.total_px, device=dev)
        self._pixstate_buf = torch.zeros(oit.PIXSTATE_PLANES * self.total_px, device=dev)
        self.image = self._image_buf
        self.pixstate = self._pixstate_buf

    def _alloc_ws(self):
        nb = oit.workspace_bytes(self.cap, self.cams_arr, self.n_views, self.tuning)
        if nb == 0:
            raise oit.OITError(oit.lib.oit_last_error().decode())
        self.ws = _aligned_workspace(nb, self.device)
        oit.clear_status(self.ws)

    def use_cameras(self, cams):
        """Point the renderer at another batch of views; the workspace and the per-pixel
        buffers grow only when the new batch needs more."""
        self.cams = list(cams)
        self.n_views = len(self.cams)
        self.cams_arr = oit.camera_array(self.cams)
        self.hw = [c.height * c.width for c in self.cams]
        self.total_px = sum(self.hw)
        nb = oit.workspace_bytes(self.cap, self.cams_arr, self.n_views, self.tuning)
        if nb == 0:
            raise oit.OITError(oit.lib.oit_last_error().decode())
        if nb > self.ws.numel():
            self._alloc_ws()
        if oit.PIXSTATE_PLANES * self.total_px > self._pixstate_buf.numel():
            self._image_buf = torch.zeros(3 * self.total_px, device=self.device)
            self._pixstate_buf = torch.zeros(oit.PIXSTATE_PLANES * self.total_px, device=self.device)
        self.image = self._image_buf[:3 * self.total_px]
        self.pixstate = self._pixstate_buf[:oit.PIXSTATE_PLANES * self.total_px]

    def set_tuning(self, tile=None, batch=None, pair_capacity=None, bwd_mode=None):
        self.tuning = oit.Tuning(int(tile or self.tuning.tile), int(batch or self.tuning.batch),
                                 int(pair_capacity or self.tuning.pair_capacity),
                                 int(self.tuning.bwd_mode if bwd_mode is None else bwd_mode), 0)
        self._alloc_ws()

    def views(self, flat: torch.Tensor, planes: int):
        """Split a packed [V][planes][H][W] buffer into per-view tensors."""
        out, o = [], 0
        for c in self.cams:
            k = planes * c.height * c.width
            out.append(flat[o:o + k].view(planes, c.height, c.width))
            o += k
        return out

    def pack(self, per_view) -> torch.Tensor:
        return torch.cat([torch.as_tensor(x, dtype=torch.float32).reshape(-1) for x in per_view]).to(
            self.device).contiguous()

    def forward(self, params, sigma, bg, active=None, pre=None, delta_params=None):
        sp = oit.splats_struct(params)
        dsp = oit.splats_struct(delta_params) if delta_params is not None else None
        a = active or {}
        oit.render_fwd(sp, sigma, bg, self.cams_arr, self.n_views, self.cap, a.get("idx"), a.get("n"),
                       a.get("delta_idx"), a.get("delta_sign"), a.get("n_delta"), pre, self.image,
                       self.pixstate, self.ws, self.tuning, delta_splats=dsp)
        return self.image

    def backward(self, params, sigma, bg, grad_image, grads, grad_sigma, active=None, pre=None, score=None,
                 eps=None):
        sp = oit.splats_struct(params)
        a = active or {}
        gs = oit.grads_struct(grads, grads["mean"].shape[1])
        oit.render_bwd(sp, sigma, bg, self.cams_arr, self.n_views, self.cap, a.get("idx"), a.get("n"),
                       a.get("delta_idx"), a.get("delta_sign"), a.get("n_delta"), pre, grad_image,
                       self.pixstate, gs, grad_sigma, score, eps, self.ws, self.tuning)

    def status(self) -> int:
        return oit.read_status(self.ws)

    def counters(self):
        return oit.read_counters(self.ws, self.cap, self.cams_arr, self.n_views, self.tuning)

    def tile_entries(self):
        """Per view, the (active, label-change) entry counts of each tile of the last
        forward: a list of [2][tiles_y][tiles_x] numpy arrays."""
        S = self.tuning.tile
        shapes = [((c.height + S - 1) // S, (c.width + S - 1) // S) for c in self.cams]
        n_tiles = sum(ty * tx for ty, tx in shapes)
        flat = oit.read_tile_entries(self.ws, self.cap, self.cams_arr, self.n_views, self.tuning, n_tiles)
        out, o = [], 0
        for ty, tx in shapes:
            out.append(flat[:, o:o + ty * tx].reshape(2, ty, tx))
            o += ty * tx
        return out

    def pairs_needed(self) -> int:
        return self.counters()[0]

    def forward_fitted(self, params, sigma, bg, active=None, pre=None, delta_params=None, slack=1.25):
        """Forward that sizes the pair capacity as it goes: one run, then (after a status
        read, which synchronises) a second one only when the tile lists overflowed.  The
        label changes are folded into the pre-rendered buffer by the run, so a copy taken
        before the first run is put back before the second."""
        folds = pre is not None and active is not None and active.get("n_delta") is not None
        backup = pre.clone() if folds else None
        self.forward(params, sigma, bg, active, pre, delta_params)
        if not self.status() & oit.STATUS_PAIR_OVERFLOW:
            return self.image
        need = self.pairs_needed()
        self.set_tuning(pair_capacity=min(int(need * slack) + 4096, 2 ** 32 - 2))
        if folds:
            pre.copy_(backup)
        return self.forward(params, sigma, bg, active, pre, delta_params)

    def fit_pair_capacity(self, params, sigma, bg, active=None, pre=None, slack=1.25, delta_params=None):
        """Run the forward once; grow the pair capacity if the tile lists overflowed."""
        pre_copy = pre.clone() if pre is not None else None
        self.forward(params, sigma, bg, active, pre_copy, delta_params)
        st = self.status()
        need = self.pairs_needed()
        if st & oit.STATUS_PAIR_OVERFLOW or need > self.tuning.pair_capacity:
            self.set_tuning(pair_capacity=min(int(need * slack) + 4096, 2 ** 32 - 2))
        return need


class PhotometricLoss:
    """The training loss: "l1" (the benchmark configurations) or "l1_dssim", the 3DGS
    loss (1 - lambda) L1 + lambda D-SSIM that the paper keeps (Sec. 5.1), lambda = 0.2.
    Owns the D-SSIM workspace and grows it with the batch."""

    def __init__(self, kind="l1", lam=0.2, device="cuda"):
        if kind not in ("l1", "l1_dssim"):
            raise ValueError(f"unknown loss {kind}")
        self.kind, self.lam, self.device = kind, float(lam), torch.device(device)
        self.ws = None

    def __call__(self, renderer, image, target, grad, loss):
        if self.kind == "l1":
            oit.l1_loss(image, target, renderer.cams_arr, renderer.n_views, grad, loss, renderer.ws)
            return
        nb = oit.loss_workspace_bytes(renderer.cams_arr, renderer.n_views)
        if self.ws is None or self.ws.numel() < nb:
            self.ws = _aligned_workspace(nb, self.device)
        oit.l1_dssim_loss(image, target, renderer.cams_arr, renderer.n_views, self.lam, grad, loss, self.ws)


def new_grads(n_rows: int, device) -> dict:
    return {g: torch.zeros((c, n_rows), device=device) for g, c in GROUPS}


class OITRender(torch.autograd.Function):
    """Dense differentiable render of a batch of views.

    forward(renderer, sigma, mean, log_scale, quat, opacity_logit, sh, vsh) -> image
    (packed [V][3][H][W]); the parameters are splat-major ([n][3], [n][3], [n][4],
    [n][1], [n][48], [n][16]).  backward returns the gradient of every parameter (same
    shapes) and of sigma.  The per-pixel totals live in the renderer between the passes.
    """

    @staticmethod
    def forward(ctx, renderer: Renderer, sigma, mean, log_scale, quat, opacity_logit, sh, vsh, bg=(0.0, 0.0, 0.0)):
        params = {"mean": mean.contiguous(), "log_scale": log_scale.contiguous(), "quat": quat.contiguous(),
                  "opacity_logit": opacity_logit.contiguous(), "sh": sh.contiguous(), "vsh": vsh.contiguous()}
        ctx.renderer = renderer
        ctx.bg = tuple(float(x) for x in bg)
        ctx.params = params
        ctx.save_for_backward(sigma)
        img = renderer.forward(params, sigma, ctx.bg)
        return img.clone()

    @staticmethod
    def backward(ctx, grad_image):
        (sigma,) = ctx.saved_tensors
        r = ctx.renderer
        grads = new_grads(r.n, sigma.device)
        gsig = torch.zeros(1, dtype=torch.float64, device=sigma.device)
        r.backward(ctx.params, sigma, ctx.bg, grad_image.contiguous(), grads, gsig)
        g = {k: t.t().contiguous() for k, t in grads.items()}   # compact [C][n] -> [n][C]
        return (None, gsig.to(sigma.dtype), g["mean"], g["log_scale"], g["quat"], g["opacity_logit"], g["sh"],
                g["vsh"], None)


def render(renderer, sigma, params, bg=(0.0, 0.0, 0.0)):
    return OITRender.apply(renderer, sigma, params["mean"], params["log_scale"], params["quat"],
                           params["opacity_logit"], params["sh"], params["vsh"], bg)


class ActiveSetTrainer:
    """Device state and the launch sequence of one training iteration."""

    def __init__(self, scene, fraction=0.05, lr=1e-3, sigma_lr=1e-3, betas=(0.9, 0.999), eps=1e-15,
                 tile=16, batch=64, pair_capacity=None, dense=False, device="cuda", delta_capacity=None,
                 loss="l1"):
        self.device = torch.device(device)
        self.loss_fn = PhotometricLoss(loss, device=device)
        dev = self.device
        self.params = params_to_device(scene.params, dev)
        self.n = self.params["mean"].shape[0]
        self.dense = dense
        self.k = self.n if dense else max(1, int(math.ceil(fraction * self.n)))
        self.bg = tuple(float(x) for x in scene.background)
        acap = self.n if dense else self.k
        dcap = 0 if dense else (self.n if delta_capacity is None else int(delta_capacity))
        self.r = Renderer(scene.cameras, self.n, acap, dcap, tile, batch, pair_capacity, dev)
        self.target = self.r.pack(scene.targets)
        self.sigma = torch.tensor([scene.sigma], dtype=torch.float32, device=dev)
        self.m = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.v = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.sig_m = torch.zeros(1, device=dev)
        self.sig_v = torch.zeros(1, device=dev)
        self.sig_step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.lr = [lr] * 6 if not isinstance(lr, (list, tuple)) else list(lr)
        self.sigma_lr = sigma_lr
        self.betas = betas
        self.eps = eps
        self.grads = new_grads(acap, dev)
        self.grad_sigma = torch.zeros(1, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.grad_image = torch.zeros(3 * self.r.total_px, device=dev)
        self.score = torch.zeros(self.n, device=dev)
        if not dense:
            self.label = torch.ones(self.n, dtype=torch.uint8, device=dev)
            self.active_idx = torch.zeros(acap, dtype=torch.int32, device=dev)
            self.n_active = torch.zeros(1, dtype=torch.int32, device=dev)
            self.delta_idx = torch.zeros(max(dcap, 1), dtype=torch.int32, device=dev)
            self.delta_sign = torch.zeros(max(dcap, 1), dtype=torch.int8, device=dev)
            self.n_delta = torch.zeros(1, dtype=torch.int32, device=dev)
            self.pre = torch.zeros(9 * self.r.total_px, device=dev)
            self.sel_ws = _aligned_workspace(oit.select_workspace_bytes(self.n), dev)
            oit.clear_status(self.sel_ws)
        self.graph = None

    # --- the pieces of one iteration -------------------------------------------------
    def _active(self):
        if self.dense:
            return None
        return {"idx": self.active_idx, "n": self.n_active, "delta_idx": self.delta_idx,
                "delta_sign": self.delta_sign, "n_delta": self.n_delta}

    def select(self):
        oit.update_active_set(self.score, self.n, oit.SELECT_TOPK, self.k, 0.0, self.label, self.active_idx,
                              self.n_active, self.delta_idx, self.delta_sign, self.n_delta, self.sel_ws)

    def forward_loss(self):
        pre = None if self.dense else self.pre
        self.r.forward(self.params, self.sigma, self.bg, self._active(), pre)
        self.loss_fn(self.r, self.r.image, self.target, self.grad_image, self.loss)

    def backward(self):
        pre = None if self.dense else self.pre
        self.r.backward(self.params, self.sigma, self.bg, self.grad_image, self.grads, self.grad_sigma,
                        self._active(), pre, self.score)

    def optimise(self):
        gs = oit.grads_struct(self.grads, self.grads["mean"].shape[1])
        idx = None if self.dense else self.active_idx
        na = None if self.dense else self.n_active
        oit.sparse_adam_step(self.params, gs, self.m, self.v, idx, na, self.n, self.lr, self.betas[0],
                             self.betas[1], self.eps, self.step)
        oit.sigma_adam_step(self.sigma, self.grad_sigma, self.sig_m, self.sig_v, self.sigma_lr, self.betas[0],
                            self.betas[1], self.eps, self.sig_step)

    def iteration(self, update_active=True):
        if not self.dense and update_active:
            self.select()
        self.forward_loss()
        self.backward()
        self.optimise()

    def warmup_dense_scores(self):
        """One untimed dense forward/backward that gives every splat a score (no update)."""
        r = Renderer(self.r.cams, self.n, self.n, 0, self.r.tuning.tile, self.r.tuning.batch, None, self.device)
        r.fit_pair_capacity(self.params, self.sigma, self.bg)
        r.forward(self.params, self.sigma, self.bg)
        gi = torch.zeros_like(self.grad_image)
        self.loss_fn(r, r.image, self.target, gi, self.loss)
        g = new_grads(self.n, self.device)
        gsig = torch.zeros(1, dtype=torch.float64, device=self.device)
        r.backward(self.params, self.sigma, self.bg, gi, g, gsig, score=self.score)
        del r

    # --- HIP graph -----------------------------------------------------------------
    def capture(self):
        """Capture one iteration into a HIP graph (state is advanced once by warm-up)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.iteration()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.iteration()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()
