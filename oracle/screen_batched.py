"""Screen the batched Riemann draws with the FP64 oracle (test infrastructure).

For each output slot, draws candidates in the slot's own order and runs each on
the oracle (one row: the problems are y-uniform) for `steps` steps; a candidate
whose solution leaves the physical range (non-finite, rho <= 0 or rho > 1e6 at
any 100-step check) is recorded as rejected and the slot draws again. The list
of rejected (slot, attempt) pairs is stored in workloads/batched_screen.json,
which the draw generator reads. Usage:

    python -m oracle.screen_batched --seed 0 --nprob 256 --steps 2000 [--jobs 8]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def physical_run(cfg, steps):
    import torch
    from oracle import scheme
    from workloads import problems as P
    c = dict(cfg, ny=1)
    pb = scheme.Problem.from_dict(c)
    f = scheme.init(pb, *P.init_fields(c))
    for n in range(steps):
        f = scheme.step(pb, f, n)
        if n % 100 == 99 or n == steps - 1:
            r = scheme.fields(pb, f)[0]
            if not bool(torch.isfinite(f).all()) or bool((r <= 0).any()) or float(r.abs().max()) > 1e6:
                return False
    return True


def screen_slot(args):
    import numpy as np
    import torch
    torch.set_num_threads(1)
    from workloads import problems as P
    seed, slot, steps, alpha, max_attempts = args
    rng = np.random.default_rng([seed, slot])
    rejected = []
    for a in range(max_attempts):
        L, left, right, st, fast, _ = P.batched_candidate(seed, slot, rng)
        cfg = P.batched_cfg(L, left, right, st, fast, steps, alpha)
        if physical_run(cfg, steps):
            return slot, rejected
        rejected.append(a)
    return slot, rejected


def main():
    from multiprocessing import Pool
    from workloads import problems as P
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--nprob", type=int, default=256)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--alpha", type=float, default=0.025)
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    jobs = [(args.seed, p, args.steps, args.alpha, 64) for p in range(args.nprob)]
    with Pool(args.jobs) as pool:
        res = pool.map(screen_slot, jobs, chunksize=1)
    rejected = sorted([slot, a] for slot, rej in res for a in rej)
    try:
        with open(P.SCREEN_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        d = {}
    d[P.screen_key(args.seed, args.steps, args.alpha)] = {
        "rejected": rejected, "nprob": args.nprob,
        "criterion": "FP64 oracle, one row, non-finite or rho <= 0 or rho > 1e6 at a 100-step check"}
    with open(P.SCREEN_FILE, "w") as fh:
        json.dump(d, fh, indent=0)
    print("rejected attempts:", len(rejected))


if __name__ == "__main__":
    main()
