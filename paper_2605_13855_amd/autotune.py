"""Autotuner for the rasteriser's tile size and LDS batch.

Candidates are timed as whole training iterations (HIP events, eager launches) on the
live trainer state, because the tile size moves work between binning, the forward
blend and the backward (bigger tiles: fewer entries, more rejected pairs per entry).
Results are cached per workload shape (splats, views, resolutions, active fraction)
in a JSON file so that a later run starts from the best known setting.
"""
from __future__ import annotations

import json
import os
import statistics

TILES = (8, 16, 32)
BATCHES = (32, 64, 128, 256)


def workload_key(trainer) -> str:
    res = ",".join(f"{c.width}x{c.height}" for c in trainer.r.cams)
    return f"n={trainer.n};k={trainer.k};dense={int(trainer.dense)};views={res}"


def load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(path, cache):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def prepare(trainer):
    """Make the trainer's tile lists fit the current tuning, then run one iteration."""
    if not trainer.dense:
        trainer.select()
        trainer.r.fit_pair_capacity(trainer.params, trainer.sigma, trainer.bg, trainer._active(), trainer.pre)
        trainer.forward_loss()
        trainer.backward()
        trainer.optimise()
    else:
        trainer.r.fit_pair_capacity(trainer.params, trainer.sigma, trainer.bg)


def time_iterations(trainer, iters=3) -> float:
    import torch
    ts = []
    for _ in range(iters):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        trainer.iteration()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return statistics.median(ts)


def autotune(trainer, tiles=TILES, batches=BATCHES, iters=3, cache_path=None, log=None):
    """Set the fastest (tile, batch) on ``trainer`` and return (best, {candidate: ms})."""
    cache = load_cache(cache_path)
    key = workload_key(trainer)
    if key in cache:
        best = tuple(cache[key]["best"])
        trainer.r.set_tuning(tile=best[0], batch=best[1])
        prepare(trainer)
        return best, {tuple(map(int, k.split("x"))): v for k, v in cache[key]["ms"].items()}
    results = {}
    for tile in tiles:
        for batch in batches:
            trainer.r.set_tuning(tile=tile, batch=batch)
            prepare(trainer)
            ms = time_iterations(trainer, iters)
            results[(tile, batch)] = ms
            if log:
                log(f"  autotune tile={tile:2d} batch={batch:3d}: {ms:8.3f} ms/iter")
    best = min(results, key=results.get)
    trainer.r.set_tuning(tile=best[0], batch=best[1])
    prepare(trainer)
    cache[key] = {"best": list(best), "ms": {f"{t}x{b}": round(v, 4) for (t, b), v in results.items()}}
    save_cache(cache_path, cache)
    return best, results
