"""The paper's active-set schedule (Sec. 4.1, Alg. "Active Set Method") on liboit.

* Every ``interval`` iterations the active set is recomputed on a subset of ``n_sub``
  training views picked by farthest-point sampling over the camera centres from a
  random start: the whole splat set is rendered on those views in one batched launch,
  the activeness score of every splat is max over attribute groups of
  ||dL/dtheta_g|| / eps_g, and the splats with score > 1 become active.
* Every iteration renders one training view (views are drawn in shuffled passes, as
  3DGS does) with the active splats against that view's pre-rendered buffer, takes the
  3DGS loss (L1 + D-SSIM by default), back-propagates to the active rows, and applies
  sparse Adam and Adam on sigma.
* Pre-rendered buffers are brought up to date lazily, when their view is next used
  (Sec. 4.1 "Implementation Details"): a buffer one update behind receives the label
  changes between its labels and the current ones in the same pass that renders it.
  The label-change splats are added and removed with their parameters as of the update
  (a snapshot taken then): a splat that became active may already have been trained
  by other views' iterations, but the buffer still holds its frozen contribution.
  A buffer two or more updates behind could hold a splat that was active and trained
  in between, so it is rebuilt from empty (all labels changing from "active").
  With ``interval`` >= 2 x views, as the paper chooses, rebuilds never happen.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import oit
from .render import PhotometricLoss, Renderer, _aligned_workspace, new_grads, params_to_device


class PaperScheduleTrainer:
    def __init__(self, scene, eps, interval=500, n_sub=30, lr=1e-3, sigma_lr=1e-3, betas=(0.9, 0.999),
                 adam_eps=1e-15, tile=16, batch=64, seed=0, device="cuda", loss="l1_dssim"):
        self.device = torch.device(device)
        self.loss_fn = PhotometricLoss(loss, device=device)
        dev = self.device
        self.params = params_to_device(scene.params, dev)
        self.n = self.params["mean"].shape[0]
        self.bg = tuple(float(x) for x in scene.background)
        self.cams = list(scene.cameras)
        self.targets = [torch.as_tensor(t, dtype=torch.float32).reshape(-1).to(dev) for t in scene.targets]
        self.centres = np.stack([c.center() for c in self.cams]).astype(np.float32)
        self.eps = [float(e) for e in eps]
        self.interval = int(interval)
        self.n_sub = min(int(n_sub), len(self.cams), oit.MAX_VIEWS)
        self.rng = np.random.default_rng(seed)
        self.lr = [lr] * 6 if not isinstance(lr, (list, tuple)) else list(lr)
        self.sigma_lr = sigma_lr
        self.betas = betas
        self.adam_eps = adam_eps
        n = self.n
        self.sigma = torch.tensor([scene.sigma], dtype=torch.float32, device=dev)
        self.m = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.snapshot = {g: t.clone() for g, t in self.params.items()}   # parameters at the last update
        self.v = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.sig_m = torch.zeros(1, device=dev)
        self.sig_v = torch.zeros(1, device=dev)
        self.sig_step = torch.zeros(1, dtype=torch.int32, device=dev)
        # labels: epoch 0 = every splat active (so every pre-rendered buffer starts empty)
        self.epoch = 0
        self.all_active = torch.ones(n, dtype=torch.uint8, device=dev)
        self.labels = {0: self.all_active.clone()}
        self.view_epoch = [0] * len(self.cams)
        self.pre = [torch.zeros(9 * c.width * c.height, device=dev) for c in self.cams]
        # buffers of the per-iteration pass
        self.active_idx = torch.zeros(n, dtype=torch.int32, device=dev)
        self.n_active = torch.zeros(1, dtype=torch.int32, device=dev)
        self.delta_idx = torch.zeros(n, dtype=torch.int32, device=dev)
        self.idx_epoch = None   # the epoch whose active list active_idx holds (None: unknown)
        self.delta_sign = torch.zeros(n, dtype=torch.int8, device=dev)
        self.n_delta = torch.zeros(1, dtype=torch.int32, device=dev)
        self.sel_ws = _aligned_workspace(oit.select_workspace_bytes(n), dev)
        self.r = Renderer([self.cams[0]], n, n, n, tile, batch, None, dev)
        self.grads = new_grads(n, dev)
        self.grad_sigma = torch.zeros(1, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.grad_image = torch.zeros(3 * max(c.width * c.height for c in self.cams), device=dev)
        # the subsampled full-set pass
        self.sub = None
        self.score = torch.zeros(n, device=dev)
        self.it = 0
        self.order = []
        self.last_update_views = []
        self.rebuilds = 0

    def update_active_set(self):
        """Activeness on FPS-subsampled views, then threshold selection (new epoch)."""
        start = int(self.rng.integers(len(self.cams)))
        views = oit.fps_views(self.centres, self.n_sub, start)
        self.last_update_views = views
        cams = [self.cams[i] for i in views]
        if self.sub is None:
            self.sub = Renderer(cams, self.n, self.n, 0, self.r.tuning.tile, self.r.tuning.batch, None, self.device)
        else:
            self.sub.use_cameras(cams)
        r = self.sub
        r.forward_fitted(self.params, self.sigma, self.bg)
        target = torch.cat([self.targets[i] for i in views])
        gi = torch.zeros_like(target)
        self.loss_fn(r, r.image, target, gi, self.loss)
        g = new_grads(self.n, self.device)
        gsig = torch.zeros(1, dtype=torch.float64, device=self.device)
        r.backward(self.params, self.sigma, self.bg, gi, g, gsig, score=self.score, eps=self.eps)
        new_label = self.labels[self.epoch].clone()
        oit.update_active_set(self.score, self.n, oit.SELECT_THRESHOLD, 0, 1.0, new_label, self.active_idx,
                              self.n_active, self.delta_idx, self.delta_sign, self.n_delta, self.sel_ws)
        self.epoch += 1
        self.labels[self.epoch] = new_label
        self.idx_epoch = self.epoch
        # every splat whose label differs between two consecutive epochs is frozen at this
        # moment: these are the values it was (or will be) added to a pre buffer with
        for g, p in self.params.items():
            self.snapshot[g].copy_(p)
        self._forget_labels()

    def _forget_labels(self):
        keep = set(self.view_epoch) | {self.epoch, 0}
        for e in list(self.labels):
            if e not in keep:
                del self.labels[e]

    def next_view(self) -> int:
        if not self.order:
            self.order = list(self.rng.permutation(len(self.cams)))
        return int(self.order.pop())

    def prepare_view(self, v):
        """Active list of the current labels and the label changes that bring view v's
        pre-rendered buffer up to date (rebuilding it if it is two updates behind)."""
        old = self.view_epoch[v]
        if old == self.epoch and self.idx_epoch == self.epoch:
            # the view's buffer is up to date and active_idx holds the current labels'
            # list: no label changes (the forward then keeps its active part's occupancy)
            return {"idx": self.active_idx, "n": self.n_active}
        if old < self.epoch - 1:
            self.pre[v].zero_()
            old_label = self.all_active
            self.rebuilds += 1
        else:
            old_label = self.labels[old]
        oit.label_delta(old_label, self.labels[self.epoch], self.n, self.active_idx, self.n_active, self.delta_idx,
                        self.delta_sign, self.n_delta, self.sel_ws)
        self.idx_epoch = self.epoch
        return {"idx": self.active_idx, "n": self.n_active, "delta_idx": self.delta_idx,
                "delta_sign": self.delta_sign, "n_delta": self.n_delta}

    def render_view(self, v, fit=True):
        """Forward of view v with the active set and its (updated) pre-rendered buffer."""
        act = self.prepare_view(v)
        self.r.use_cameras([self.cams[v]])
        if fit:
            self.r.forward_fitted(self.params, self.sigma, self.bg, act, self.pre[v], self.snapshot)
        else:
            self.r.forward(self.params, self.sigma, self.bg, act, self.pre[v], self.snapshot)
        self.view_epoch[v] = self.epoch
        self._forget_labels()
        return act

    def iteration(self, fit=True):
        """One training iteration on the next view.  fit=False skips the status read that
        grows the pair capacity on overflow (the caller then checks the status word)."""
        if self.it % self.interval == 0:
            self.update_active_set()
        v = self.next_view()
        act = self.render_view(v, fit)
        gi = self.grad_image[:3 * self.cams[v].width * self.cams[v].height]
        self.loss_fn(self.r, self.r.image, self.targets[v], gi, self.loss)
        self.r.backward(self.params, self.sigma, self.bg, gi, self.grads, self.grad_sigma, act, self.pre[v])
        gs = oit.grads_struct(self.grads, self.n)
        oit.sparse_adam_step(self.params, gs, self.m, self.v, self.active_idx, self.n_active, self.n, self.lr,
                             self.betas[0], self.betas[1], self.adam_eps, self.step)
        oit.sigma_adam_step(self.sigma, self.grad_sigma, self.sig_m, self.sig_v, self.sigma_lr, self.betas[0],
                            self.betas[1], self.adam_eps, self.sig_step)
        self.it += 1
        return v

    def active_fraction(self) -> float:
        return float(self.labels[self.epoch].float().mean().item())
