#!/usr/bin/env python
"""Benchmark of one SparseOIT training iteration on one MI355X.

Workload (default): 1,000,000 splats, 16 views of uneven size (640x480 .. 1600x1200)
on an orbit of radius 4, 5% of the splats active (top-k of the activeness score every
step), L1 loss, sparse Adam.  One step = active-set selection + forward (projection,
tile binning, blend-and-normalise with the pre-rendered inactive set and its update)
+ loss + backward + sparse Adam + Adam on sigma, captured once as a HIP graph and
replayed.  The dense full-set form of the same iteration is measured beside it.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32, 256 CUs x 2.4 GHz x 256 flop/clk
PEAK_HBM_GBS = 8000.0
# algorithmic flops per (splat, pixel) pair, an FMA counting 2.  Evaluated pair: the
# exponent's column and row terms and the threshold test.  Forward, contributing: exp,
# cap, alpha w, three P FMAs, the Q add, the dQ/dsigma FMA, the T update.  Backward,
# contributing: A.c - s1, three dL/dc FMAs, dL/dw and its lambda-weighted sum (for
# dL/dsigma), dL/dalpha = B / (1 - alpha) + w (A.c - s1), dL/de, the six
# exponent-gradient FMAs and dL/dmean'.
FWD_FLOP_EVAL, FWD_FLOP_CONTRIB = 10, 14
BWD_FLOP_EVAL, BWD_FLOP_CONTRIB = 10, 41


KERNEL_SOURCES = {
    "k_raster_bwd": ("k_backward.hip", "oit_device.h", "oit_internal.h"),
    "k_raster_fwd": ("k_forward.hip", "oit_device.h", "oit_internal.h"),
}


def kernel_source_hash(kname):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kname]:
        with open(os.path.join(ROOT, "paper_2605_13855_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_traffic(kname, tile, batch):
    """HBM bytes per launch of `kname` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (profiles/<kname>_traffic.txt, or profiles/<kname>_traffic_batch<B>.txt for
    the forward at another LDS batch), or None when there is none for this tiling or the
    kernel's sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kname}_traffic.txt")
    if kname == "k_raster_fwd":
        per_batch = os.path.join(ROOT, "profiles", f"{kname}_traffic_batch{batch}.txt")
        if os.path.exists(per_batch):
            path = per_batch
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    try:
        if fields.get("source_sha256") != kernel_source_hash(kname):
            return None
        # the backward kernel does not depend on the forward's staging batch
        if int(fields["tile"]) != tile or (kname == "k_raster_fwd" and int(fields["batch"]) != batch):
            return None
        return int(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic HBM bytes per unit of each stage (float32 data; N splats, V views, R listed
# records = active rows + label changes, E tile entries of the call, px pixels):
#   select          6 B per splat (score read, label read and written) + 4 B per active
#                   index + 5 B per label change
#   preprocess      300 B of parameters per listed record + 60 B per (record, view):
#                   the 48-byte record, its tile rectangle and hit count
#   binning         40 B per tile entry: the list's key, slot and record written and the
#                   stable sort's passes over them
#   raster fwd      52 B per entry (index and record staged per tile) + 36 B per pixel
#                   (image and pixel state written); bound by the FP32 VALU, whose work
#                   is 10 flops per evaluated (splat, pixel) pair + 14 per contributing
#                   one (the label changes' blends are not counted)
#   loss            36 B per pixel (image and target read, dL/dC written)
#   pixel consts    60 B per pixel (state and dL/dC read, constants written), +32 B with
#                   a pre-rendered buffer
#   raster bwd      104 B per entry (index, slot, record, partials row) + 24 B per pixel
#                   (constants); VALU: 10 flops per evaluated pair + 41 per contributing
#   preprocess bwd  44 B per entry (partials row) + 604 B per active row (parameters
#                   read, gradients and score written)
#   adam            2100 B per active row (parameters, gradient, both moments)
def stage_work(run, n, views, px, dense):
    """{stage: (bound, algorithmic bytes or flops)} of one step of `run`."""
    k = run["active"]
    d = run["kernel_deltas"]
    rec = k + d
    e = run["kernel_entries"]
    ev, pc = run["kernel_evals"], run["kernel_pairs"]
    w = {"preprocess": ("hbm", 300.0 * rec + 60.0 * rec * views),
         "binning": ("hbm", 40.0 * e),
         "raster_fwd": ("alu", ev * FWD_FLOP_EVAL + pc * FWD_FLOP_CONTRIB),
         "loss": ("hbm", 36.0 * px),
         "pixconst": ("hbm", (60.0 if dense else 92.0) * px),
         "raster_bwd": ("alu", ev * BWD_FLOP_EVAL + pc * BWD_FLOP_CONTRIB),
         "preprocess_bwd": ("hbm", 44.0 * e + 604.0 * k),
         "adam": ("hbm", 2100.0 * k)}
    if not dense:
        w["select"] = ("hbm", 6.0 * n + 4.0 * k + 5.0 * d)
    return w


def stage_roofs(run, n, views, px, dense):
    """Each stage's time (eager timing pass, median) and its fraction of its binding roof."""
    out = {}
    for name, (bound, work) in stage_work(run, n, views, px, dense).items():
        ms = run["stages_ms"].get(name)
        if ms is None or ms <= 0:
            continue
        rate = work / (ms * 1e-3)
        if bound == "hbm":
            out[name] = {"ms": round(ms, 4), "bound": "hbm", "alg_bytes": work,
                         "GB_s": round(rate / 1e9, 1), "frac": round(rate / 1e9 / PEAK_HBM_GBS, 4)}
        else:
            out[name] = {"ms": round(ms, 4), "bound": "alu", "alg_flops": work,
                         "TFLOP_s": round(rate / 1e12, 2), "frac": round(rate / 1e12 / PEAK_FP32_TFLOPS, 4)}
    return out


def step_bytes(run, n, views, px, dense):
    """Algorithmic HBM bytes of one whole step (every stage's, the raster stages' bytes
    included) and its FP32 flops."""
    e = run["kernel_entries"]
    tot, flops = 0.0, 0.0
    for name, (bound, work) in stage_work(run, n, views, px, dense).items():
        if bound == "hbm":
            tot += work
        else:
            flops += work
    tot += 52.0 * e + 36.0 * px + 104.0 * e + 24.0 * px
    return tot, flops


def prime(trainer):
    """First iterations, eager, with the pair capacity fitted before each; returns the
    largest number of tile entries they needed.  In the active form the first selection
    moves every splat outside the new active set out of the label set, so that step's
    tile lists are dense-sized; the second is a steady-state step."""
    from paper_2605_13855_amd import oit
    need = 0
    for _ in range(1 if trainer.dense else 2):
        if not trainer.dense:
            trainer.select()
            trainer.r.fit_pair_capacity(trainer.params, trainer.sigma, trainer.bg, trainer._active(), trainer.pre)
        else:
            trainer.r.fit_pair_capacity(trainer.params, trainer.sigma, trainer.bg)
        trainer.forward_loss()
        trainer.backward()
        trainer.optimise()
        need = max(need, trainer.r.pairs_needed())
        st = trainer.r.status()
        if st & oit.STATUS_PAIR_OVERFLOW:
            raise RuntimeError("pair capacity overflow after fitting")
    return need


def timed_iteration(t):
    """One eager iteration with events at the boundaries of the ABI calls (select, render
    forward, loss, render backward, Adam); with the library's timing on, the render calls
    also record their inner stages.  Returns {stage: ms}."""
    import torch
    from paper_2605_13855_amd import oit
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    if not t.dense:
        t.select()
    ev[1].record()
    pre = None if t.dense else t.pre
    t.r.forward(t.params, t.sigma, t.bg, t._active(), pre)
    ev[2].record()
    t.loss_fn(t.r, t.r.image, t.target, t.grad_image, t.loss)
    ev[3].record()
    t.backward()
    ev[4].record()
    t.optimise()
    ev[5].record()
    torch.cuda.synchronize()
    out = oit.timing_read_stages()
    out["select"] = ev[0].elapsed_time(ev[1])
    out["loss"] = ev[2].elapsed_time(ev[3])
    out["adam"] = ev[4].elapsed_time(ev[5])
    out["forward_call"] = ev[1].elapsed_time(ev[2])
    out["backward_call"] = ev[3].elapsed_time(ev[4])
    return out


def run_form(scene, dense, steps, warmup, fraction, tile, batch, tune, eager=False, late_gap=0):
    """Time one form of the step.  The autotuner, if asked, runs on a throwaway trainer,
    so the timed trainer starts from the same state with or without it.  Graph replays
    (or eager steps) give the step time; a short eager pass after them times the
    raster kernels with start/stop events that bracket exactly the kernel (events
    recorded inside a captured graph do not wait for the preceding kernel)."""
    import torch
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd.render import ActiveSetTrainer

    name = "dense" if dense else f"active {fraction:.0%}"
    tuned = None
    if tune:
        from paper_2605_13855_amd.autotune import autotune
        log(f"{name}: autotune")
        t = ActiveSetTrainer(scene, fraction=fraction, tile=tile, batch=batch, dense=dense)
        if not dense:
            t.warmup_dense_scores()
        prime(t)
        (tile, batch), res = autotune(t, log=log)
        tuned = {"tile": tile, "batch": batch, "candidates_ms": {f"{k[0]}x{k[1]}": round(v, 4) for k, v in res.items()}}
        del t
        torch.cuda.empty_cache()
    log(f"{name}: building trainer")
    t = ActiveSetTrainer(scene, fraction=fraction, tile=tile, batch=batch, dense=dense)
    if not dense:
        t.warmup_dense_scores()
    need = prime(t)
    # headroom for the tile lists of later steps (the active set moves); the binning's
    # work follows the entries, not the capacity
    t.r.set_tuning(pair_capacity=min(int(need * 1.5) + 65536, 2 ** 32 - 2))
    log(f"{name}: tile={t.r.tuning.tile} batch={t.r.tuning.batch} pair_capacity={t.r.tuning.pair_capacity}")
    step = t.iteration if eager else t.replay
    if not eager:
        t.capture()
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    oit.clear_status(t.r.ws)
    log(f"{name}: timing {steps} {'eager steps' if eager else 'graph replays'}")
    def timed_window():
        """`steps` timed steps; per step its time, label changes and the counters."""
        w = {k: [] for k in ("ms", "deltas", "entries", "pairs", "evals", "chunks", "boxes", "waves")}
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            step()
            e1.record()
            torch.cuda.synchronize()
            w["ms"].append(e0.elapsed_time(e1))
            if not t.dense:
                w["deltas"].append(int(t.n_delta.item()))
            c = t.r.counters()
            for key, x in zip(("entries", "pairs", "evals", "chunks", "boxes", "waves"), c):
                w[key].append(x)
        return w

    win = timed_window()
    step_ms, pairs, evals, entries, chunks, boxes, waves = (win[k] for k in ("ms", "pairs", "evals", "entries",
                                                                             "chunks", "boxes", "waves"))
    deltas = win["deltas"]
    # kernel timing pass: eager steps with kernel-bracketing events, and the pair
    # counters of the same launches
    ksteps = max(3, steps // 2)
    oit.timing_enable(True)
    fwd_ms, bwd_ms, kpairs, kevals, kentries, kdeltas, stage_ms = [], [], [], [], [], [], []
    for _ in range(ksteps):
        stage_ms.append(timed_iteration(t))
        f, b = oit.timing_read()
        fwd_ms.append(f)
        bwd_ms.append(b)
        kdeltas.append(0 if t.dense else int(t.n_delta.item()))
        c = t.r.counters()
        kentries.append(c[0])
        kpairs.append(c[1])
        kevals.append(c[2])
    oit.timing_enable(False)
    torch.cuda.synchronize()
    stages = {k: statistics.median(d[k] for d in stage_ms) for k in stage_ms[0]}
    late = None
    if late_gap > 0:
        # a later window of the same run: the active set keeps moving as training goes on
        for _ in range(late_gap):
            step()
        torch.cuda.synchronize()
        lw = timed_window()
        late = {"after_steps": warmup + steps + ksteps + late_gap, "ms_per_step": round(statistics.mean(lw["ms"]), 4),
                "ms_median": round(statistics.median(lw["ms"]), 4),
                "contributing_pairs": statistics.mean(lw["pairs"]), "tile_entries": statistics.mean(lw["entries"])}
        if lw["deltas"]:
            late["label_changes_per_step"] = round(statistics.mean(lw["deltas"]), 1)
        log(f"{name}: late window after {late['after_steps']} steps: {late['ms_per_step']:.3f} ms/step")
    st = t.r.status()
    if st:
        raise RuntimeError(f"device status {st} during the timed steps")
    loss = float(t.loss.item())
    out = {
        "ms_per_step": statistics.mean(step_ms),
        "ms_per_step_median": statistics.median(step_ms),
        "raster_fwd_ms": statistics.mean(fwd_ms),
        "raster_bwd_ms": statistics.mean(bwd_ms),
        "kernel_steps": ksteps,
        "kernel_pairs": statistics.mean(kpairs),
        "kernel_evals": statistics.mean(kevals),
        "kernel_entries": statistics.mean(kentries),
        "kernel_deltas": statistics.mean(kdeltas),
        "stages_ms": stages,
        "label_changes": deltas,
        "late": late,
        "pairs": statistics.mean(pairs),
        "evals": statistics.mean(evals),
        "entries": statistics.mean(entries),
        "chunks": statistics.mean(chunks),
        "box_items": statistics.mean(boxes),
        "wave_items": statistics.mean(waves),
        "loss": loss,
        "active": t.k,
        "tile": t.r.tuning.tile,
        "batch": t.r.tuning.batch,
        "tuned": tuned,
    }
    log(f"{name}: {out['ms_per_step']:.3f} ms/step; raster fwd {out['raster_fwd_ms']:.3f} ms, "
        f"bwd {out['raster_bwd_ms']:.3f} ms per launch; {out['pairs']:.3e} contributing pairs")
    del t
    torch.cuda.empty_cache()
    return out


def tile_skew(scene, fraction, tile, batch, steps):
    """Entries per tile of the forward (one workgroup per tile): per view the mean and
    the largest count, for the active form after `steps` training steps (active entries
    and label changes) and for the dense form; and the bound that the heaviest tile puts
    on a launch's tail, max / (total / resident workgroups)."""
    import numpy as np
    import torch
    from paper_2605_13855_amd.render import ActiveSetTrainer
    out = {}
    for name, dense in (("active", False), ("dense", True)):
        t = ActiveSetTrainer(scene, fraction=fraction, tile=tile, batch=batch, dense=dense)
        if not dense:
            t.warmup_dense_scores()
        need = prime(t)
        t.r.set_tuning(pair_capacity=min(int(need * 1.5) + 65536, 2 ** 32 - 2))
        for _ in range(steps if not dense else 1):
            t.iteration()
        torch.cuda.synchronize()
        views = t.r.tile_entries()
        per_view, allw = [], []
        for k, v in enumerate(views):
            a, d = v[0].astype(np.float64), v[1].astype(np.float64)
            w = a + d
            allw.append(w.ravel())
            per_view.append({"view": k, "tiles": int(w.size), "active_mean": round(float(a.mean()), 1),
                             "active_max": int(a.max()), "changes_mean": round(float(d.mean()), 1),
                             "changes_max": int(d.max()), "max_over_mean": round(float(w.max() / max(w.mean(), 1e-9)), 2)})
        w = np.concatenate(allw)
        resident = 256 * 7   # workgroups of the forward at tile 32 (seven waves per SIMD, four per block)
        out[name] = {"views": per_view, "tiles": int(w.size), "entries": int(w.sum()),
                     "mean": round(float(w.mean()), 1), "max": int(w.max()),
                     "max_over_mean": round(float(w.max() / max(w.mean(), 1e-9)), 2),
                     "tail_bound": round(float(w.max() / max(w.sum() / resident, 1e-9)), 3)}
        log(f"tile skew {name}: mean {out[name]['mean']}, max {out[name]['max']}, tail bound {out[name]['tail_bound']}")
        del t
        torch.cuda.empty_cache()
    return out


def ablation(scene, steps, tile, batch):
    """Synthetic analogue of the paper's backward ablation (Tab. "ablation"): the dense
    iteration with the per-splat backward against the per-pixel backward that adds an
    atomic per contributing pair (the 3DGS design), on the same tile lists."""
    import torch
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd.render import ActiveSetTrainer
    out = {}
    for name, mode in (("per_splat", oit.BWD_PER_SPLAT), ("per_pixel_atomics", oit.BWD_PER_PIXEL)):
        t = ActiveSetTrainer(scene, tile=tile, batch=batch, dense=True)
        t.r.set_tuning(bwd_mode=mode)
        prime(t)
        oit.timing_enable(True)
        ms, bwd = [], []
        for _ in range(steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            t.iteration()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
            bwd.append(oit.timing_read()[1])
        oit.timing_enable(False)
        out[name] = {"ms_per_iter": round(statistics.median(ms), 4), "raster_bwd_ms": round(statistics.median(bwd), 4)}
        log(f"ablation {name}: {out[name]}")
        del t
        torch.cuda.empty_cache()
    out["bwd_speedup_per_splat"] = round(out["per_pixel_atomics"]["raster_bwd_ms"] / out["per_splat"]["raster_bwd_ms"], 3)
    return out


def schedule_bench(scene, iters, interval, fraction, tile, batch):
    """The paper's schedule (Sec. 4.1): one training view per iteration, the active set
    recomputed every `interval` iterations on FPS-subsampled views with an epsilon
    threshold (chosen here from the scores so that about `fraction` of the splats are
    active), L1 + D-SSIM; and the same loop with every splat active beside it."""
    import numpy as np
    import torch
    from paper_2605_13855_amd.schedule import PaperScheduleTrainer

    nv = len(scene.cameras)
    probe = PaperScheduleTrainer(scene, eps=[1.0] * 6, interval=interval, n_sub=nv, tile=tile, batch=batch)
    probe.update_active_set()
    eps = [float(np.quantile(probe.score.cpu().numpy(), 1.0 - fraction))] * 6
    del probe
    torch.cuda.empty_cache()
    out = {}
    for name, e in (("active", eps), ("all_active", [1e-30] * 6)):
        t = PaperScheduleTrainer(scene, eps=e, interval=interval, n_sub=nv, tile=tile, batch=batch)
        for _ in range(nv):          # one pass over the views grows the capacities
            t.iteration()
        torch.cuda.synchronize()
        ms, fracs = [], [round(t.active_fraction(), 4)]
        for _ in range(iters):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            upd = t.it % interval == 0
            e0.record()
            t.iteration()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
            if upd:
                fracs.append(round(t.active_fraction(), 4))
        upd = [m for i, m in enumerate(ms) if (nv + i) % interval == 0]
        out[name] = {"ms_per_iter": round(statistics.mean(ms), 4), "ms_median": round(statistics.median(ms), 4),
                     "update_iters_ms": [round(x, 3) for x in upd], "active_fraction_per_update": fracs,
                     "rebuilds": t.rebuilds}
        log(f"schedule {name}: {out[name]}")
        del t
        torch.cuda.empty_cache()
    out["speedup"] = round(out["all_active"]["ms_per_iter"] / out["active"]["ms_per_iter"], 3)
    return out


def densify_bench(scene, iters, interval, keep_probability, tile, batch, fraction=0.1):
    """The first training phase (3DGS-style, with the paper's random keep probability,
    Sec. 5.1): one view per iteration, dense forward / L1 + D-SSIM / backward, the
    densification statistic every iteration, densify-and-prune every `interval`
    iterations.  The gradient threshold is set from the statistic after one pass over
    the views so that `fraction` of the visible splats reach it (3DGS's 0.0002 is tuned
    to photographs; on these synthetic scenes no splat reaches it).  Reports the
    iteration time with and without a densification, the statistic kernel alone and
    the splat count."""
    import torch
    from paper_2605_13855_amd import oit
    from paper_2605_13855_amd.density import DensifyingTrainer

    t = DensifyingTrainer(scene, densify_from=0, densify_until=10 ** 9, densify_interval=interval,
                          opacity_reset_interval=10 ** 9, keep_probability=keep_probability, tile=tile, batch=batch)
    for _ in range(len(scene.cameras)):      # one pass grows the pair capacity
        t.iteration()
    torch.cuda.synchronize()
    seen = t.control.denom > 0
    avg = (t.control.accum[seen] / t.control.denom[seen]).double()
    thr = float(torch.quantile(avg[torch.randperm(avg.numel(), device=avg.device)[:1 << 20]], 1.0 - fraction))
    t.control.rules["grad_threshold"] = thr
    plain, dens, counts = [], [], [t.n]
    for _ in range(iters):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        before = len(t.history)
        e0.record()
        t.iteration()
        e1.record()
        torch.cuda.synchronize()
        (dens if len(t.history) > before else plain).append(e0.elapsed_time(e1))
        if len(t.history) > before:
            counts.append(t.n)
    # the statistic kernel alone, on the last backward's workspace
    stat = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        t.control.accumulate(t.r)
        e1.record()
        torch.cuda.synchronize()
        stat.append(e0.elapsed_time(e1))
    out = {"iter_ms_median": round(statistics.median(plain), 4), "iter_ms_mean": round(statistics.mean(plain), 4),
           "densify_iter_ms": [round(x, 2) for x in dens], "stats_kernel_ms": round(statistics.median(stat), 4),
           "splats": counts, "interval": interval, "keep_probability": keep_probability,
           "grad_threshold": thr, "candidate_fraction": fraction}
    log(f"densify: {out}")
    return out


_CPU_SCENE = None   # the scene the oracle workers read (set before they are forked)


def _oracle_window(win):
    """The FP64 oracle's forward and backward on one window of view 0, all splats
    (dL/dC random inside the window); returns (contributing pairs, seconds)."""
    import numpy as np
    from oracle import oracle as O
    sc = _CPU_SCENE
    cam = sc.cameras[0]
    x0, y0, x1, y1 = win
    t0 = time.perf_counter()
    r = O.render(sc.params, sc.sigma, sc.background, cam, window=win)
    g = np.zeros((3, cam.height, cam.width))
    g[:, y0:y1, x0:x1] = np.random.default_rng(x0 * 7919 + y0).normal(size=(3, y1 - y0, x1 - x0))
    O.backward(sc.params, sc.sigma, sc.background, cam, g, window=win)
    return r["pairs"], time.perf_counter() - t0


def cpu_baseline(scene, budget_s=20.0):
    """The FP64 oracle as it stands (single-threaded C), fwd + bwd on windows of view 0
    with all splats: first one process on a centre window sized to about half the
    budget, then one process per host core (at most 16, the box's share) on a grid of
    windows around the centre, run at once.  Runs before the GPU is touched: the
    workers are forked."""
    import multiprocessing as mp
    global _CPU_SCENE
    _CPU_SCENE = scene
    cam = scene.cameras[0]
    cx, cy = cam.width // 2, cam.height // 2
    side = 48
    while True:
        win = (cx - side // 2, cy - side // 2, cx + side // 2, cy + side // 2)
        pairs1, dt1 = _oracle_window(win)
        log(f"cpu oracle, 1 core: window {side}x{side}: {pairs1:.3e} pairs, {dt1:.2f} s")
        if dt1 > budget_s / 2 or side >= min(512, cam.width, cam.height) - 1:
            break
        # the work grows with the window area; aim the next window at the budget
        side = min(512, cam.width, cam.height, int(side * math.sqrt(budget_s / max(dt1, 1e-3))))
        side -= side % 2
    single = {"value": pairs1 / dt1, "cores": 1,
              "sample": f"centre window {side}x{side}: {pairs1} contributing pairs in {dt1:.2f} s"}
    cores = min(len(os.sched_getaffinity(0)), 16)
    cols = math.ceil(math.sqrt(cores))
    rows = math.ceil(cores / cols)
    ps = min(side, cam.width // cols, cam.height // rows)
    ps -= ps % 2
    gx0, gy0 = cx - cols * ps // 2, cy - rows * ps // 2
    wins = [(gx0 + (i % cols) * ps, gy0 + (i // cols) * ps, gx0 + (i % cols + 1) * ps, gy0 + (i // cols + 1) * ps)
            for i in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_window, wins)
    wall = time.perf_counter() - t0
    pairs = sum(r[0] for r in res)
    log(f"cpu oracle, {cores} cores: {cores} windows {ps}x{ps}: {pairs:.3e} pairs, {wall:.2f} s")
    return {"value": pairs / wall, "unit": "splat-pixel evals/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle fwd+bwd, view 0 ({cam.width}x{cam.height}), all {scene.n} splats: "
                      f"{cores} processes on a {cols}x{rows} grid of {ps}x{ps} windows around the centre, "
                      f"{pairs} contributing pairs in {wall:.2f} s wall",
            "single_core": single}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--fraction", type=float, default=0.05)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--log-scale-mu", type=float, default=-3.5)
    ap.add_argument("--eager", action="store_true", help="launch every step eagerly instead of a HIP graph")
    ap.add_argument("--ablation", action="store_true",
                    help="instead of the benchmark line, time the per-splat against the per-pixel backward "
                         "(dense; default config 2)")
    ap.add_argument("--schedule", action="store_true",
                    help="instead of the benchmark line, time the paper's active-set schedule (one view per "
                         "iteration, FPS-subsampled threshold updates, L1 + D-SSIM) against all splats active")
    ap.add_argument("--interval", type=int, default=50,
                    help="active-set update interval for --schedule, densification interval for --densify")
    ap.add_argument("--densify", action="store_true",
                    help="instead of the benchmark line, time the first training phase with densification")
    ap.add_argument("--keep-probability", type=float, default=0.5, help="densification keep probability (--densify)")
    ap.add_argument("--tile-skew", action="store_true",
                    help="instead of the benchmark line, report the forward's entries per tile (active and dense)")
    ap.add_argument("--late-gap", type=int, default=100,
                    help="untimed steps between the timed window and a second, later timed window (0: none)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is "
              f"described, not built", file=sys.stderr)
        sys.exit(2)

    from paper_2605_13855_amd import scenes
    bench_line = not (args.ablation or args.densify or args.schedule or args.tile_skew)
    scene = cpu = None
    if bench_line:
        log(f"building scene config {args.config}")
        scene = scenes.make_scene(args.config, log_scale_mu=args.log_scale_mu)
        # the oracle's workers are forked before anything touches the GPU
        cpu = None if args.no_cpu else cpu_baseline(scene)

    import torch
    from paper_2605_13855_amd import oit  # noqa: F401  (fails loudly without the HIP library)

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_mb:
        nel = args.copy_mb * (1 << 20) // 4
        src = torch.ones(nel, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.copy_mb} MiB read + {args.copy_mb} MiB written")
        del src, dst
    if args.ablation:
        cfg = args.config if "--config" in sys.argv else 2
        scene = scenes.make_scene(cfg)
        res = ablation(scene, args.steps, args.tile, args.batch)
        print(json.dumps({"ablation": res, "config": {"workload": f"config {cfg}: {scene.n} splats, "
                          f"{len(scene.cameras)} view(s), dense fwd+bwd, L1"}}), flush=True)
        return
    if args.tile_skew:
        scene = scenes.make_scene(args.config, log_scale_mu=args.log_scale_mu)
        res = tile_skew(scene, args.fraction, args.tile, args.batch, args.steps)
        print(json.dumps({"tile_skew": res, "config": {
            "workload": f"config {args.config}: {scene.n} splats, {len(scene.cameras)} views, "
                        f"{args.fraction:.0%} active after {args.steps} steps; dense",
            "tile": args.tile, "batch": args.batch}}), flush=True)
        return
    if args.densify:
        scene = scenes.make_scene(args.config, log_scale_mu=args.log_scale_mu)
        res = densify_bench(scene, args.steps, args.interval, args.keep_probability, args.tile, args.batch,
                            args.fraction)
        print(json.dumps({"densify": res, "config": {
            "workload": f"config {args.config}: {scene.n} splats at the start, {len(scene.cameras)} views, one view "
                        f"per iteration, densify and prune every {args.interval} iterations (3DGS rules, keep "
                        f"probability {args.keep_probability}), L1 + D-SSIM", "tile": args.tile, "batch": args.batch}}),
              flush=True)
        return
    if args.schedule:
        scene = scenes.make_scene(args.config, log_scale_mu=args.log_scale_mu)
        res = schedule_bench(scene, args.steps, args.interval, args.fraction, args.tile, args.batch)
        print(json.dumps({"schedule": res, "config": {
            "workload": f"config {args.config}: {scene.n} splats, {len(scene.cameras)} views, one view per "
                        f"iteration, update every {args.interval} iterations on all views (FPS), "
                        f"~{args.fraction:.0%} active, L1 + D-SSIM", "tile": args.tile, "batch": args.batch}}),
              flush=True)
        return
    px = sum(c.width * c.height for c in scene.cameras)
    log(f"scene: {scene.n} splats, {len(scene.cameras)} views, {px} pixels")

    act = run_form(scene, False, args.steps, args.warmup, args.fraction, args.tile, args.batch,
                   not args.no_autotune, args.eager, late_gap=args.late_gap)
    dense = None
    if not args.no_dense:
        dense = run_form(scene, True, max(3, args.steps // 4), max(1, args.warmup // 2), 1.0, act["tile"],
                         act["batch"], False, args.eager)

    # dominant kernel of the active step, roofline against the FP32 vector peak; flops
    # from the pair counters of the launches that were timed
    fwd_flops = act["kernel_evals"] * FWD_FLOP_EVAL + act["kernel_pairs"] * FWD_FLOP_CONTRIB
    bwd_flops = act["kernel_evals"] * BWD_FLOP_EVAL + act["kernel_pairs"] * BWD_FLOP_CONTRIB
    if act["raster_bwd_ms"] >= act["raster_fwd_ms"]:
        kname, kms, kflops = "k_raster_bwd", act["raster_bwd_ms"], bwd_flops
    else:
        kname, kms, kflops = "k_raster_fwd", act["raster_fwd_ms"], fwd_flops
    achieved = kflops / (kms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": committed_traffic(kname, act["tile"], act["batch"]),
                "flops_per_launch": kflops, "avg_launch_ms": round(kms, 4), "timed_launches": act["kernel_steps"]}
    value = act["pairs"] / (act["ms_per_step"] * 1e-3)
    nv = len(scene.cameras)
    line = {
        "metric": "fwd+bwd ms/iter and splat-pixel evals/s, active-set vs dense, 1M splats",
        "value": value,
        "unit": "splat-pixel evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(act["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "launch": "eager" if args.eager else "hipGraph",
        "data": "synthetic",
        "config": {
            "workload": f"config {args.config}: {scene.n} splats, {len(scene.cameras)} views "
                        f"({px} px, uneven 640x480..1600x1200), {args.fraction:.0%} active top-k each step, "
                        f"hipGraph iteration, L1 + sparse Adam",
            "splats": scene.n, "views": len(scene.cameras), "pixels": px, "active_fraction": args.fraction,
            "tile": act["tile"], "batch": act["batch"], "log_scale_mu": args.log_scale_mu,
        },
        "active": {"ms_per_step": round(act["ms_per_step"], 4), "ms_median": round(act["ms_per_step_median"], 4),
                   "evals_per_s": value, "contributing_pairs": act["pairs"], "evaluated_pairs": act["evals"],
                   "tile_entries": act["entries"], "bwd_work_items": act["chunks"], "bwd_box_items": act["box_items"],
                   "bwd_wave_items": act["wave_items"],
                   "raster_fwd_ms": round(act["raster_fwd_ms"], 4), "raster_bwd_ms": round(act["raster_bwd_ms"], 4),
                   "label_changes_per_step": {"mean": round(statistics.mean(act["label_changes"]), 1),
                                              "min": min(act["label_changes"]), "max": max(act["label_changes"])},
                   "late_window": act["late"],
                   "stages": stage_roofs(act, scene.n, nv, px, False),
                   "loss": act["loss"], "autotune": act["tuned"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if dense is not None:
        line["dense"] = {"ms_per_step": round(dense["ms_per_step"], 4),
                         "evals_per_s": dense["pairs"] / (dense["ms_per_step"] * 1e-3),
                         "contributing_pairs": dense["pairs"], "evaluated_pairs": dense["evals"],
                         "tile_entries": dense["entries"], "bwd_work_items": dense["chunks"],
                         "bwd_box_items": dense["box_items"], "bwd_wave_items": dense["wave_items"],
                         "raster_fwd_ms": round(dense["raster_fwd_ms"], 4),
                         "raster_bwd_ms": round(dense["raster_bwd_ms"], 4),
                         "stages": stage_roofs(dense, scene.n, nv, px, True)}
        db, dflops = step_bytes(dense, scene.n, nv, px, True)
        rate = db / (dense["ms_per_step"] * 1e-3) / 1e9
        line["dense"]["hbm"] = {"alg_bytes_per_step": db, "GB_s": round(rate, 1),
                                "hbm_frac": round(rate / PEAK_HBM_GBS, 4),
                                "alg_flops_per_step": dflops,
                                "valu_frac": round(dflops / (dense["ms_per_step"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)}
        line["speedup_active_vs_dense"] = round(dense["ms_per_step"] / act["ms_per_step"], 3)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
