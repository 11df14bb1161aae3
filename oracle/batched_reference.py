"""Reference results of the batched Riemann workload from the oracle (test
infrastructure; writes tests/golden/batched_reference.npz).

For each of the 256 problems of the batched workload (seed 0, 2000 steps, one
row: the problems are uniform in y on a periodic 4-row grid):
  * the density after 2000 steps of the FP64 oracle (scheme.run),
  * the density after 2000 steps with FP32 storage (every stored state rounded to
    float32, the arithmetic of each step in float64: scheme.run(storage=float32)),
  * the von Neumann chooser of Sec. 3: the largest candidate alpha = c2 dt/dx
    (workloads VN_ALPHAS) such that it and every smaller candidate keep the
    spectral radius of G(k) (Eqs. (SEC-VON-8), (SEC-VON-9), (SEC-VON-12)) at most
    1 + VN_TOL at the problem's left, right and two star states over the wave
    vectors of workloads.vn_wave_vectors, with the largest radius at that alpha
    and at the next candidate.
Usage: python -m oracle.batched_reference [--jobs 8]
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(ROOT, "tests", "golden", "batched_reference.npz")
STEPS = 2000


def one_problem(k):
    import torch
    torch.set_num_threads(1)
    from oracle import scheme, vonneumann as ovn
    from workloads import problems as P
    cfgs, _ = P.batched(nprob=256, seed=0, steps=STEPS)
    c1 = dict(cfgs[k], ny=1)
    pb = scheme.Problem.from_dict(c1)
    f0 = scheme.init(pb, *P.init_fields(c1))
    r64 = scheme.fields(pb, scheme.run(pb, f0, STEPS))[0][0]
    f32 = scheme.store(f0, torch.float32)
    r32 = scheme.fields(pb, scheme.run(pb, f32, STEPS, storage=torch.float32))[0][0]
    kx, ky = P.vn_wave_vectors()
    chosen, r_at, r_next = None, 0.0, 0.0
    for st in P.batched_vn_states(cfgs[k]):
        J = ovn.collision_jacobian(*st, pb.c1, pb.c2, pb.eta0, pb.gamma)
        last, rl, rn = 0.0, 0.0, 0.0
        for a in P.VN_ALPHAS:
            prm = {"c1": pb.c1, "c2": pb.c2, "eta0": pb.eta0, "gamma": pb.gamma, "tau": pb.tau, "beta": pb.beta,
                   "dt": a * pb.dx / pb.c2, "dx": pb.dx, "lam": pb.lam}
            r = ovn.max_modulus_many(st, prm, kx, ky, J)
            if r > 1.0 + P.VN_TOL:
                rn = r
                break
            last, rl = a, r
        if chosen is None or last < chosen:
            chosen = last
        # radii of the deciding state: largest passing radius at the chosen alpha, smallest failing
        r_at = max(r_at, rl)
        r_next = rn if r_next == 0.0 else (min(r_next, rn) if rn > 0.0 else r_next)
    return k, r64.numpy(), r32.numpy(), chosen, r_at, r_next


def main():
    import numpy as np
    from multiprocessing import Pool
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    with Pool(args.jobs) as pool:
        res = sorted(pool.map(one_problem, range(256), chunksize=1), key=lambda r: r[0])
    lengths = np.array([len(r[1]) for r in res], dtype=np.int64)
    np.savez_compressed(
        OUT, steps=np.int64(STEPS), lengths=lengths,
        rho64=np.concatenate([r[1] for r in res]),
        drho32=np.concatenate([(r[2] - r[1]).astype(np.float32) for r in res]),
        rel_l1_fp32_storage=np.array([np.abs(r[2] - r[1]).sum() / np.abs(r[1]).sum() for r in res]),
        alpha_vn=np.array([r[3] for r in res]), radius_at_alpha=np.array([r[4] for r in res]),
        radius_next_alpha=np.array([r[5] for r in res]))
    print("wrote", OUT, "problems", len(res), "cells", int(lengths.sum()))


if __name__ == "__main__":
    main()
