"""Checkpoint and resume of the trainers (``DensifyingTrainer``, ``PaperScheduleTrainer``,
``ActiveSetTrainer``).

A checkpoint is one safetensors file: every device tensor of the trainer's state (splat
parameters, Adam moments and step counters, sigma and its Adam state, and per trainer
the densification statistic and its random generator, or the label arrays, the
per-view pre-rendered buffers and the parameter snapshot), plus JSON metadata for the
host state (iteration counters, the view order, the numpy generator, pair capacity).
Loading restores into a trainer built for the same scene; its splat count may differ
(densification), so the trainer's buffers are rebuilt to the checkpoint's size.  The
kernels are deterministic (no order-dependent sums), so a resumed run repeats the
uninterrupted one bit for bit.
"""
from __future__ import annotations

import json

import numpy as np
import torch
from safetensors.torch import load_file, save_file

from . import oit
from .render import GROUPS, new_grads

FORMAT = "oit-checkpoint-1"


def _host(t: torch.Tensor) -> torch.Tensor:
    return t.detach().contiguous().cpu().clone()


def _groups(prefix, d, out):
    for g, _ in GROUPS:
        out[f"{prefix}/{g}"] = _host(d[g])


def _common(t, out):
    _groups("params", t.params, out)
    _groups("m", t.m, out)
    _groups("v", t.v, out)
    for k in ("step", "sigma", "sig_m", "sig_v", "sig_step"):
        out[k] = _host(getattr(t, k))


def state(trainer):
    """(tensors, metadata) of a trainer."""
    from .density import DensifyingTrainer
    from .render import ActiveSetTrainer
    from .schedule import PaperScheduleTrainer

    tensors, meta = {}, {"format": FORMAT}
    _common(trainer, tensors)
    if isinstance(trainer, DensifyingTrainer):
        c = trainer.control
        tensors["control/accum"] = _host(c.accum)
        tensors["control/denom"] = _host(c.denom)
        tensors["control/max_radius"] = _host(c.max_radius)
        tensors["control/generator"] = c.gen.get_state().clone()
        meta.update(kind="densify", it=trainer.it, order=[int(x) for x in trainer.order],
                    history=[list(h) for h in trainer.history], rng=trainer.rng.bit_generator.state,
                    pair_capacity=int(trainer.r.tuning.pair_capacity))
    elif isinstance(trainer, PaperScheduleTrainer):
        _groups("snapshot", trainer.snapshot, tensors)
        for e, lab in trainer.labels.items():
            tensors[f"labels/{e}"] = _host(lab)
        for i, p in enumerate(trainer.pre):
            tensors[f"pre/{i}"] = _host(p)
        meta.update(kind="schedule", it=trainer.it, epoch=trainer.epoch, view_epoch=list(trainer.view_epoch),
                    order=[int(x) for x in trainer.order], last_update_views=[int(x) for x in trainer.last_update_views],
                    rebuilds=trainer.rebuilds, rng=trainer.rng.bit_generator.state,
                    pair_capacity=int(trainer.r.tuning.pair_capacity))
    elif isinstance(trainer, ActiveSetTrainer):
        for k in ("label", "score", "pre"):
            if hasattr(trainer, k):
                tensors[k] = _host(getattr(trainer, k))
        meta.update(kind="active")
    else:
        raise TypeError(f"no checkpoint format for {type(trainer).__name__}")
    return tensors, meta


def save(trainer, path):
    tensors, meta = state(trainer)
    save_file(tensors, str(path), metadata={"oit": json.dumps(meta)})


def _restore_groups(prefix, dst: dict, src: dict, device):
    for g, _ in GROUPS:
        dst[g] = src[f"{prefix}/{g}"].to(device).contiguous()


def load(trainer, path):
    """Restore a checkpoint into ``trainer`` (built for the same scene and kind)."""
    from safetensors import safe_open

    with safe_open(str(path), framework="pt") as f:
        meta = json.loads(f.metadata()["oit"])
    if meta.get("format") != FORMAT:
        raise ValueError(f"{path}: not an {FORMAT} file")
    t = load_file(str(path))
    dev = trainer.device
    kind = meta["kind"]
    want = {"densify": "DensifyingTrainer", "schedule": "PaperScheduleTrainer", "active": "ActiveSetTrainer"}[kind]
    if type(trainer).__name__ != want:
        raise TypeError(f"{path} holds a {want} state, not a {type(trainer).__name__} one")
    if kind == "active":
        for g, _ in GROUPS:
            trainer.params[g].copy_(t[f"params/{g}"])
            trainer.m[g].copy_(t[f"m/{g}"])
            trainer.v[g].copy_(t[f"v/{g}"])
        for k in ("step", "sigma", "sig_m", "sig_v", "sig_step", "label", "score", "pre"):
            if k in t:
                getattr(trainer, k).copy_(t[k])
        return trainer
    _restore_groups("params", trainer.params, t, dev)
    _restore_groups("m", trainer.m, t, dev)
    _restore_groups("v", trainer.v, t, dev)
    for k in ("step", "sigma", "sig_m", "sig_v", "sig_step"):
        setattr(trainer, k, t[k].to(dev))
    rng = np.random.default_rng()
    rng.bit_generator.state = meta["rng"]
    trainer.rng = rng
    trainer.it = int(meta["it"])
    trainer.order = [int(x) for x in meta["order"]]
    if kind == "densify":
        trainer.history = [tuple(h) for h in meta["history"]]
        c = trainer.control
        c.reset(trainer.n)
        c.accum.copy_(t["control/accum"])
        c.denom.copy_(t["control/denom"])
        c.max_radius.copy_(t["control/max_radius"])
        c.gen.set_state(t["control/generator"])
        trainer._build()
    else:
        n = trainer.n
        if int(t["params/mean"].shape[0]) != n:
            raise ValueError("the schedule trainer keeps its splat count: build it for the checkpoint's scene")
        _restore_groups("snapshot", trainer.snapshot, t, dev)
        trainer.labels = {int(k.split("/")[1]): t[k].to(dev) for k in t if k.startswith("labels/")}
        for i in range(len(trainer.pre)):
            trainer.pre[i].copy_(t[f"pre/{i}"])
        trainer.epoch = int(meta["epoch"])
        trainer.view_epoch = [int(x) for x in meta["view_epoch"]]
        trainer.last_update_views = [int(x) for x in meta["last_update_views"]]
        trainer.rebuilds = int(meta["rebuilds"])
        trainer.idx_epoch = None   # active_idx is not in the checkpoint: the next view rebuilds it
        trainer.grads = new_grads(n, dev)
    cap = int(meta["pair_capacity"])
    if cap > trainer.r.tuning.pair_capacity:
        trainer.r.set_tuning(pair_capacity=cap)
    oit.clear_status(trainer.r.ws)
    return trainer
