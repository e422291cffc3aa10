"""The first training phase with density control, and the hand-over to the active-set
schedule.

The paper trains its first 15,000 iterations as 3DGS does, with 3DGS's densification
and pruning plus a scene-specific random keep probability that caps the splat count,
and switches to the active-set method afterwards (Sec. 5.1 "Implementation Details";
Fig. "overview").  The rules live with ``oit_densify_plan`` in ``include/oit.h``.

* ``DensityControl`` owns the per-splat statistic (summed screen-space mean gradient
  norm, visible views, largest screen radius) and runs plan / apply on the device; the
  random draws come from a seeded ``torch.Generator`` on the device.
* ``DensifyingTrainer`` is the first phase: one training view per iteration (shuffled
  passes), dense forward / loss / backward, Adam on every splat and on sigma, the
  statistic accumulated inside the densification window, densify-and-prune every
  ``densify_interval`` iterations and an opacity reset every ``opacity_reset_interval``.
  The screen-size and world-size pruning start after the first opacity reset, as in
  3DGS.  Learning-rate decay schedules are not modelled.
* ``hand_over`` starts the paper's active-set schedule from the first phase's splats,
  Adam moments and sigma.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import oit
from .render import GROUPS, PhotometricLoss, Renderer, _aligned_workspace, new_grads, params_to_device


def scene_extent(cams) -> float:
    """3DGS's scene radius: 1.1 x the largest distance of a camera centre from their mean."""
    c = np.stack([cam.center() for cam in cams])
    return float(1.1 * np.linalg.norm(c - c.mean(axis=0), axis=1).max())


class DensityControl:
    def __init__(self, n, rules: dict, device="cuda", seed=0):
        self.device = torch.device(device)
        self.rules = dict(rules)
        self.gen = torch.Generator(device=self.device)
        self.gen.manual_seed(int(seed))
        self.reset(n)

    def reset(self, n):
        self.n = int(n)
        self.accum = torch.zeros(self.n, device=self.device)
        self.denom = torch.zeros(self.n, device=self.device)
        self.max_radius = torch.zeros(self.n, device=self.device)

    def accumulate(self, r: Renderer):
        """Add the statistic of the renderer's last (dense) backward."""
        oit.densify_stats(r.cams_arr, r.n_views, r.cap, None, None, None, self.accum, self.denom, self.max_radius,
                          r.ws, r.tuning)

    def rules_struct(self, **override) -> oit.DensityRules:
        d = {**self.rules, **override}
        return oit.DensityRules(float(d["grad_threshold"]), float(d["percent_dense"]), float(d["scene_extent"]),
                                float(d["min_opacity"]), float(d.get("max_screen_size", 0.0)),
                                float(d.get("max_world_frac", 0.0)), float(d.get("keep_probability", 1.0)), 0)

    def densify(self, params: dict, m: dict, v: dict, **override):
        """Densify and prune; returns the new (params, m, v) and resets the statistic."""
        n = self.n
        uniform = torch.rand(n, device=self.device, generator=self.gen)
        normals = torch.randn((n, 2, 3), device=self.device, generator=self.gen)
        ws = _aligned_workspace(oit.densify_workspace_bytes(n), self.device)
        n_new = torch.zeros(1, dtype=torch.int64, device=self.device)
        sp = oit.splats_struct(params)
        oit.densify_plan(sp, self.accum, self.denom, self.max_radius, uniform, self.rules_struct(**override), n_new,
                         ws)
        nn = int(n_new.item())
        if nn <= 0:
            raise RuntimeError("densification pruned every splat")
        p2 = {g: torch.empty((nn, c), device=self.device) for g, c in GROUPS}
        m2 = {g: torch.empty((nn, c), device=self.device) for g, c in GROUPS}
        v2 = {g: torch.empty((nn, c), device=self.device) for g, c in GROUPS}
        oit.densify_apply(sp, m, v, normals, p2, m2, v2, nn, ws)
        self.reset(nn)
        return p2, m2, v2


class DensifyingTrainer:
    def __init__(self, scene, lr=None, sigma_lr=0.1, betas=(0.9, 0.999), adam_eps=1e-15, densify_from=500,
                 densify_until=15000, densify_interval=100, opacity_reset_interval=3000, grad_threshold=0.0002,
                 percent_dense=0.01, min_opacity=0.005, keep_probability=1.0, tile=16, batch=64, seed=0,
                 device="cuda", loss="l1_dssim"):
        self.device = torch.device(device)
        dev = self.device
        self.cams = list(scene.cameras)
        self.bg = tuple(float(x) for x in scene.background)
        self.targets = [torch.as_tensor(t, dtype=torch.float32).reshape(-1).to(dev) for t in scene.targets]
        self.extent = scene_extent(self.cams)
        # the paper's rates for opacity, sigma and v; 3DGS's for the rest (no decay)
        self.lr = lr or [1.6e-4 * self.extent, 5e-3, 1e-3, 1e-2, 2.5e-3, 5e-3]
        self.sigma_lr, self.betas, self.adam_eps = sigma_lr, betas, adam_eps
        self.densify_from, self.densify_until = densify_from, densify_until
        self.densify_interval, self.reset_interval = densify_interval, opacity_reset_interval
        self.params = params_to_device(scene.params, dev)
        self.m = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.v = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.sigma = torch.tensor([scene.sigma], dtype=torch.float32, device=dev)
        self.sig_m = torch.zeros(1, device=dev)
        self.sig_v = torch.zeros(1, device=dev)
        self.sig_step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss_fn = PhotometricLoss(loss, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.grad_sigma = torch.zeros(1, dtype=torch.float64, device=dev)
        self.grad_image = torch.zeros(3 * max(c.width * c.height for c in self.cams), device=dev)
        self.tile, self.batch = tile, batch
        self.control = DensityControl(self.n, dict(grad_threshold=grad_threshold, percent_dense=percent_dense,
                                                   scene_extent=self.extent, min_opacity=min_opacity,
                                                   keep_probability=keep_probability), dev, seed)
        self.rng = np.random.default_rng(seed)
        self.order = []
        self.it = 0
        self.history = []   # (iteration, splats after) of every densification
        self._build()

    @property
    def n(self) -> int:
        return int(self.params["mean"].shape[0])

    def _build(self):
        cap = None if not hasattr(self, "r") else self.r.tuning.pair_capacity
        self.r = Renderer([self.cams[0]], self.n, self.n, 0, self.tile, self.batch, cap, self.device)
        self.grads = new_grads(self.n, self.device)

    def next_view(self) -> int:
        if not self.order:
            self.order = list(self.rng.permutation(len(self.cams)))
        return int(self.order.pop())

    def in_window(self) -> bool:
        return self.densify_from <= self.it < self.densify_until

    def iteration(self):
        v = self.next_view()
        cam = self.cams[v]
        self.r.use_cameras([cam])
        self.r.forward_fitted(self.params, self.sigma, self.bg)
        gi = self.grad_image[:3 * cam.width * cam.height]
        self.loss_fn(self.r, self.r.image, self.targets[v], gi, self.loss)
        self.r.backward(self.params, self.sigma, self.bg, gi, self.grads, self.grad_sigma)
        if self.in_window():
            self.control.accumulate(self.r)
        gs = oit.grads_struct(self.grads, self.n)
        oit.sparse_adam_step(self.params, gs, self.m, self.v, None, None, self.n, self.lr, self.betas[0],
                             self.betas[1], self.adam_eps, self.step)
        oit.sigma_adam_step(self.sigma, self.grad_sigma, self.sig_m, self.sig_v, self.sigma_lr, self.betas[0],
                            self.betas[1], self.adam_eps, self.sig_step)
        self.it += 1
        if self.in_window() and self.it > self.densify_from and self.it % self.densify_interval == 0:
            self.densify_and_prune()
        if self.it < self.densify_until and self.it % self.reset_interval == 0:
            self.reset_opacity()
        return v

    def densify_and_prune(self):
        big = self.it > self.reset_interval
        self.params, self.m, self.v = self.control.densify(
            self.params, self.m, self.v, max_screen_size=20.0 if big else 0.0, max_world_frac=0.1 if big else 0.0)
        self.history.append((self.it, self.n))
        self._build()

    def reset_opacity(self, max_opacity=0.01):
        oit.reset_opacity(self.params["opacity_logit"], self.m["opacity_logit"], self.v["opacity_logit"], self.n,
                          max_opacity)


class _SceneView:
    """The fields of a scene that the schedule trainer reads, over host arrays."""

    def __init__(self, cams, targets, background, params, sigma):
        self.cameras, self.targets, self.background = cams, targets, background
        self.params, self.sigma = params, sigma


def hand_over(first: DensifyingTrainer, scene, eps, **kw):
    """The active-set schedule, started from the first phase's splats, Adam moments
    and sigma (the paper switches at the end of densification, Sec. 5.1)."""
    from .render import params_to_host
    from .schedule import PaperScheduleTrainer

    view = _SceneView(scene.cameras, scene.targets, scene.background, params_to_host(first.params),
                      float(first.sigma.item()))
    t = PaperScheduleTrainer(view, eps, **kw)
    for g in t.params:
        t.params[g].copy_(first.params[g])
        t.snapshot[g].copy_(first.params[g])
        t.m[g].copy_(first.m[g])
        t.v[g].copy_(first.v[g])
    t.step.copy_(first.step)
    t.sigma.copy_(first.sigma)
    t.sig_m.copy_(first.sig_m)
    t.sig_v.copy_(first.sig_v)
    t.sig_step.copy_(first.sig_step)
    return t
