"""Launch-shape autotuner with an on-disk cache.

Single grid: lb_autotune times every (block_x, rows, blocks) candidate, one step
per launch and two steps per pass, with HIP events on the real grid. Batched: each block_x candidate of the packed work list is
timed over a few graph-launched steps. Results are cached in a JSON file keyed
by device name, precision and shape, so later runs reuse them.
"""
from __future__ import annotations

import json
import os

import torch

from . import api

CACHE = os.environ.get("LBKT_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(d):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _key(kind, prec, shape):
    return "%s|%s|%s|%s" % (torch.cuda.get_device_name(0), kind, prec, shape)


def tile_for(grid: api.Grid, f_a, f_b, prec="f64", reps=10, refresh=False):
    """Best (block_x, rows, blocks, steps_per_pass) of lb_run for this grid shape
    (pass it as lb.run(..., tile=...)); f_a/f_b are overwritten."""
    d = _load()
    k = _key("step", prec, "%dx%d" % (grid.nx, grid.ny))
    if k in d and not refresh:
        return tuple(d[k]["tile"])
    tile, ms = api.autotune(grid, f_a, f_b, prec=prec, reps=reps)
    d[k] = {"tile": list(tile), "ms": ms}
    _store(d)
    return tile


def batch_block_for(batch: api.Batch, f_a, f_b, steps=200, refresh=False, reps=3):
    """Best block_x for a batch (f_a/f_b are overwritten); applies it to the batch.
    Each width is timed as the median of `reps` graph launches of `steps` steps
    (the widths differ by a few percent, less than one short launch varies)."""
    sig = "%d:%d" % (len(batch.grids), sum(g.nx * g.ny for g in batch.grids))
    d = _load()
    k = _key("batched", "f64" if batch.prec == 0 else "f32", sig)
    if k in d and not refresh:
        batch.set_tile(d[k]["block_x"])
        return d[k]["block_x"]
    best, best_ms = None, None
    s = torch.cuda.current_stream()
    for bx in (64, 128, 256):
        batch.set_tile(bx)
        batch.step(f_a, f_b, steps)            # capture
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            batch.step(f_a, f_b, steps)
            e1.record(s)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = sorted(times)[len(times) // 2]
        if best_ms is None or ms < best_ms:
            best, best_ms = bx, ms
    batch.set_tile(best)
    d[k] = {"block_x": best, "ms": best_ms, "steps": steps}
    _store(d)
    return best
