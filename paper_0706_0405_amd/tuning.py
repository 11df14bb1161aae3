"""Launch-shape autotuner with an on-disk cache.

Single grid: lb_autotune times every (block_x, rows, blocks) candidate, one step
per launch and two steps per pass, with HIP events on the real grid. Batched: each block_x candidate of the packed work list is
timed over a few graph-launched steps. Results are cached in a JSON file keyed
by device name, precision and shape, so later runs reuse them.
"""
from __future__ import annotations

import json
import os
import time

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


def batch_block_for(batch: api.Batch, f_a, f_b, steps=200, refresh=False, reps=3, settle_ms=250.0):
    """Best block_x for a batch (f_a/f_b are overwritten); applies it to the batch.
    The widths are timed in `reps` interleaved rounds (one graph launch of `steps`
    steps each, after an untimed launch that captures it), after untimed launches
    that keep the GPU busy for settle_ms (clocks ramp up after an idle period);
    the median per width decides (the widths differ by a few percent)."""
    sig = "%d:%d" % (len(batch.grids), sum(g.nx * g.ny for g in batch.grids))
    d = _load()
    k = _key("batched", "f64" if batch.prec == 0 else "f32", sig)
    if k in d and not refresh:
        batch.set_tile(d[k]["block_x"])
        return d[k]["block_x"]
    widths = (64, 128, 256)
    s = torch.cuda.current_stream()
    batch.set_tile(widths[0])
    t0 = time.perf_counter()
    n = 0
    while n < 2 or (time.perf_counter() - t0) * 1e3 < settle_ms:
        batch.step(f_a, f_b, steps)
        torch.cuda.synchronize()
        n += 1
    times = {bx: [] for bx in widths}
    for _ in range(reps):
        for bx in widths:
            batch.set_tile(bx)
            batch.step(f_a, f_b, steps)            # capture (untimed)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            batch.step(f_a, f_b, steps)
            e1.record(s)
            torch.cuda.synchronize()
            times[bx].append(e0.elapsed_time(e1))
    med = {bx: sorted(v)[len(v) // 2] for bx, v in times.items()}
    best = min(widths, key=lambda bx: med[bx])
    batch.set_tile(best)
    d[k] = {"block_x": best, "ms": med[best], "steps": steps, "ms_by_width": {str(b): m for b, m in med.items()}}
    _store(d)
    return best
