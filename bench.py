#!/usr/bin/env python3
"""Benchmark of the FDLB D2V9 step on one MI355X.

One step = one time step of the finite-difference lattice Boltzmann scheme
(moments, f_eq, beta-mixed upwind convection, dissipation, BGK relaxation and
update) over the whole grid, through the C ABI. The workload is the
double-Mach-reflection field on an 8192 x 2048 grid (a 1.2 GB FP64 / 0.6 GB FP32
array, too large for the 256 MB on-chip cache), timed as a HIP-graph replay of
K steps of lb_run with HIP events on the stream that runs the kernels.

Prints ONE JSON line: MLUPS of lb_run for FP64 storage (value: two time steps per
pass over the array, its default), the same for FP32 storage, and one step per
launch (the single fused step kernel) for both, each against the HBM roofline
of its kernel; the batched-problem speedup; the adjoint / forward time ratio;
and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# --profile-run: every leg with minimal repetition (one timed replay, no settle, no
# one-at-a-time comparison), for rocprofv3 counter passes, which serialise dispatches
PROFILE = False
BYTES_PER_SITE = {"f64": 144, "f32": 72}   # 9 loads + 9 stores of the storage type per pass


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in ("paper_0706_0405_amd/csrc/lbkt.hip", "paper_0706_0405_amd/csrc/kt_site.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, prec):
    """HBM bytes per launch of `kernel` ("k_step", "k_step2" or "k_step3") from a committed
    rocprofv3 counter summary, if it was taken from the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", "traffic_step_roofline_grid.txt")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(kernel, {}).get(prec)
    if not e or d.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def fields_to(dev, fields):
    import numpy as np
    import torch
    return [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev) for a in fields]


def replays(s, replay, settle_ms=250.0, reps=7):
    """Time `reps` calls of replay() (each one graph replay, or one fixed batch of
    launches, on stream s), each bracketed by HIP events and a device
    synchronisation, after untimed calls that keep the GPU busy for at least
    settle_ms (the first work after the GPU has idled runs up to 20% slower while
    its clocks come up). Returns the per-call times in ms (in call order)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    while n < 2 or (time.perf_counter() - t0) * 1e3 < settle_ms:
        replay()
        torch.cuda.synchronize()
        n += 1
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        replay()
        e1.record(s)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def median(v):
    w = sorted(v)
    return w[len(w) // 2] if len(w) % 2 else 0.5 * (w[len(w) // 2 - 1] + w[len(w) // 2])


def spread(v):
    """min / median / max of a list of times and the relative range."""
    m = median(v)
    return {"min": min(v), "median": m, "max": max(v), "rel_range": (max(v) - min(v)) / m, "n": len(v)}


def time_step(prec, steps, warmup, dev, per_pass=2, long_ms=20.0):
    """lb_run on the roofline grid with `per_pass` time steps per launch (steps a
    multiple of 12, so that a run is all passes of per_pass steps): W warm-up steps,
    the K-step graph captured, then the median of 7 replays of exactly K steps
    (after the settle replays); as a check, the median of 5 replays of a graph of
    K_long >= K steps lasting at least long_ms each."""
    import torch
    import paper_0706_0405_amd as lb
    from workloads import problems as P

    cfg = P.roofline_grid()
    g = lb.Grid.from_workload(cfg)
    rho, ux, uy, p = fields_to(dev, P.init_fields(cfg))
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        fa = lb.init(g, rho, ux, uy, p, prec=prec)
        fb = lb.empty(g, prec, dev)
        del rho, ux, uy, p
        if warmup > 0:
            lb.run(g, fa, fb, warmup, prec=prec, steps_per_pass=per_pass)
        run_k = lambda: lb.run(g, fa, fb, steps, prec=prec, use_graph=True, steps_per_pass=per_pass)  # noqa: E731
        run_k()   # capture (untimed)
        times = replays(s, run_k, **({"settle_ms": 0.0, "reps": 1} if PROFILE else {}))
        ms = median(times)
        k_long = steps * max(1, math.ceil(long_ms / ms))   # a multiple of 4: the result stays in fa
        if PROFILE:
            k_long, long_times = steps, times
        else:
            run_long = lambda: lb.run(g, fa, fb, k_long, prec=prec, use_graph=True, steps_per_pass=per_pass)  # noqa: E731
            run_long()
            long_times = replays(s, run_long, settle_ms=0.0, reps=5)
        _, _, _, _, flags = lb.moments(g, fa, prec=prec)
        torch.cuda.synchronize()
    sites = g.nx * g.ny
    launches = steps // per_pass
    per_launch_ms = ms / launches
    mlups = sites * steps / (ms * 1e-3) / 1e6
    long_mlups = sites * k_long / (median(long_times) * 1e-3) / 1e6
    achieved = BYTES_PER_SITE[prec] * sites / (per_launch_ms * 1e-3) / 1e9
    kname = {1: "k_step", 2: "k_step2", 3: "k_step3"}[per_pass]
    traffic = measured_traffic(kname, prec)
    # the one-step HBM bound on the update rate: peak / (bytes per site per step)
    bound_mlups = HBM_PEAK_GBS * 1e9 / BYTES_PER_SITE[prec] / 1e6
    res = {
        "mlups": mlups, "ms_per_step": ms / steps, "steps_per_pass": per_pass, "grid": [g.nx, g.ny],
        "flags": [int(v) for v in flags.cpu().tolist()],
        "mlups_vs_one_step_hbm_bound": mlups / bound_mlups,
        "replays": {"steps_each": steps, "ms": spread(times),
                    "check_long": {"steps_each": k_long, "ms": spread(long_times), "mlups": long_mlups,
                                   "ratio_to_value": long_mlups / mlups}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname if per_pass == 3 else "%s<%s>" % (kname, "double" if prec == "f64" else "float"),
                     "launch_ms": per_launch_ms,
                     "algorithmic_bytes_per_launch": BYTES_PER_SITE[prec] * sites},
    }
    del fa, fb
    torch.cuda.empty_cache()
    return res


def copy_bandwidth(dev, nbytes=9 * 2048 * 8192 * 8, reps=20):
    """Device-to-device copy of an array the size of the FP64 distribution array
    (torch's copy kernel): the bandwidth a plain streaming kernel reaches here."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def bench_batched(dev, steps=2000, nprob=256):
    """cfg: 256 Riemann problems of uneven length, FP32 storage, one graph launch of
    `steps` steps (the library's default for 4-row y-periodic batches: four steps
    per pass, each strip's state in registers) vs the sum of single-problem lb_run
    runs (its default on these grids: sixteen steps per pass) and vs the plain
    single-problem step (one step per launch); and the same batch in FP64 storage
    at its default eight steps per pass against two."""
    import torch
    import paper_0706_0405_amd as lb
    from workloads import problems as P

    if PROFILE:
        steps = 8   # two deep passes of four steps (the default depth in FP32 storage)
    cfgs, info = P.batched(nprob=nprob, seed=0, steps=steps)
    grids = [lb.Grid.from_workload(c) for c in cfgs]
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        B = lb.Batch(grids, "f32")
        fa, fb = B.empty(dev), B.empty(dev)
        fa.zero_()
        fb.zero_()

        def init_all():
            for k, (c, g) in enumerate(zip(cfgs, grids)):
                rho, ux, uy, p = fields_to(dev, P.init_fields(c))
                lb.init(g, rho, ux, uy, p, prec="f32", out=B.view(fa, k))

        from paper_0706_0405_amd import tuning
        init_all()
        if PROFILE:   # one replay at every block width (the tuner's candidates), the last one 256
            for bx in (64, 128, 256):
                B.set_tile(bx)
                init_all()
                B.step(fa, fb, steps)
            block_x = 256
        else:
            block_x = tuning.batch_block_for(B, fa, fb)   # block width chosen by timing (cached per device)
        init_all()
        f_init = fa.clone()

        def replay():   # from the initial fields: a device copy, then the graph launch
            fa.copy_(f_init)
            return B.step(fa, fb, steps)

        replay()                        # capture + first replay (untimed)
        # timed replays after a settle phase (the copy before each is outside the
        # events: they are recorded behind it on the same stream)
        times = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        while not PROFILE and (time.perf_counter() - t0) < 0.25:
            replay()
            torch.cuda.synchronize()
        for _ in range(1 if PROFILE else 5):
            fa.copy_(f_init)
            e0.record(s)
            out = B.step(fa, fb, steps)
            e1.record(s)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        t_batch = median(times)
        del f_init
        nonfinite = 0
        for k, g in enumerate(grids):
            _, _, _, _, fl = lb.moments(g, B.view(out, k), prec="f32")
            nonfinite += int(int(fl[1]) > 0)
        # the same problems one at a time: lb_run's default, and one step per launch
        t_single = 0.0
        t_one = 0.0
        for k, (c, g) in enumerate(zip(cfgs, grids) if not PROFILE else ()):
            rho, ux, uy, p = fields_to(dev, P.init_fields(c))
            f1 = lb.init(g, rho, ux, uy, p, prec="f32")
            f2 = lb.empty(g, "f32", dev)
            f1_0 = f1.clone()
            torch.cuda.synchronize()
            e0.record(s)
            lb.run(g, f1, f2, steps, prec="f32", steps_per_pass=1)
            e1.record(s)
            torch.cuda.synchronize()
            t_one += e0.elapsed_time(e1)
            f1.copy_(f1_0)
            torch.cuda.synchronize()
            e0.record(s)
            r = lb.run(g, f1, f2, steps, prec="f32")
            e1.record(s)
            torch.cuda.synchronize()
            t_single += e0.elapsed_time(e1)
            if k < 8:   # the packed result is bitwise the single-problem result (NaNs included)
                a = r[:, :, :g.nx].contiguous().view(torch.int32)
                b = B.view(out, k)[:, :, :g.nx].contiguous().view(torch.int32)
                if not torch.equal(a, b):
                    raise RuntimeError("batched result differs from the single-problem run (problem %d)" % k)
        B.close()
        # the same batch in double storage: the default 8 steps per pass (a strip's
        # whole state in registers) against 2, bitwise the same result
        f64 = None
        if not PROFILE:
            B = lb.Batch(grids, "f64")
            fa, fb = B.empty(dev), B.empty(dev)
            fa.zero_()
            fb.zero_()
            for k, (c, g) in enumerate(zip(cfgs, grids)):
                lb.init(g, *fields_to(dev, P.init_fields(c)), prec="f64", out=B.view(fa, k))
            f0 = fa.clone()
            f64 = {}
            outs = []
            for name, spp in (("default", 0), ("two_steps_per_pass", 2)):
                B.set_tile(64, spp)
                fa.copy_(f0)
                outs.append(B.step(fa, fb, steps).clone())
                f64[name + "_ms"] = median(replays(s, lambda: B.step(fa, fb, steps), reps=3))
            f64["steps_per_pass"] = 8
            f64["bitwise_equal"] = bool(torch.equal(outs[0].view(torch.int64), outs[1].view(torch.int64)))
            B.close()
            del fa, fb, f0, outs
    sites = sum(g.nx * g.ny for g in grids)
    mlups = sites * steps / (t_batch * 1e-3) / 1e6
    return {"problems": nprob, "steps": steps, "sites": sites, "draws": info, "block_x": block_x,
            "batched_ms": t_batch, "batched_ms_replays": spread(times),
            "single_sum_ms": t_single, "speedup": t_single / t_batch if t_single else None,
            "single_one_step_per_launch_sum_ms": t_one,
            "speedup_vs_one_step_per_launch": t_one / t_batch if t_one else None,
            "batched_mlups": mlups, "steps_per_pass": 4,
            "mlups_vs_one_step_hbm_bound": mlups * 1e6 * BYTES_PER_SITE["f32"] / (HBM_PEAK_GBS * 1e9),
            "nonfinite_problems": nonfinite, "f64_storage": f64}


def bench_adjoint_step(dev, fwd_ms, nsteps=20):
    """One adjoint step (k_adjoint, FP32 f, FP64 g) on the roofline grid, per launch, against the
    FP32-storage forward step on the same grid: 36 + 72 + 72 = 180 algorithmic bytes per site."""
    import torch
    import paper_0706_0405_amd as lb
    from paper_0706_0405_amd import api
    from workloads import problems as P

    cfg = P.roofline_grid()
    g = lb.Grid.from_workload(cfg)
    rho, ux, uy, p = fields_to(dev, P.init_fields(cfg))
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        f = lb.init(g, rho, ux, uy, p, prec="f32")
        del rho, ux, uy, p
        ga = lb.empty(g, "f64", dev)
        ga.normal_()
        gb = lb.empty(g, "f64", dev)
        if PROFILE:
            nsteps = 2
        states = [f] * nsteps   # nsteps adjoint steps, direct launches (no graph)
        times = replays(s, lambda: api.adjoint_run(g, states, ga, gb, prec="f32"),
                        **({"settle_ms": 0.0, "reps": 1} if PROFILE else {}))
        out = ga if nsteps % 2 == 0 else gb
        ms = median(times) / nsteps
        finite = bool(torch.isfinite(out[:, :, :g.nx]).all())
        del f, ga, gb, out, states
    torch.cuda.empty_cache()
    sites = g.nx * g.ny
    achieved = 180 * sites / (ms * 1e-3) / 1e9
    return {"grid": [g.nx, g.ny], "kernel": "k_adjoint<float>", "ms_per_step": ms,
            "replays_ms": spread([t / nsteps for t in times]),
            "mlups": sites / (ms * 1e-3) / 1e6, "forward_ms_per_step": fwd_ms,
            "ratio": ms / fwd_ms if fwd_ms else None,
            "ratio_by_bytes": 180 / 72, "achieved_gbs": achieved, "roofline_frac": achieved / HBM_PEAK_GBS,
            "finite": finite}


def vn_cases():
    """The chooser's inputs for the 256 batched Riemann problems (as in the oracle's
    reference): each problem's left, right and two star states as cases, the candidate
    time steps alpha dx / c2, the owning problem, and the 64 x 4 wave vectors of a
    4-row periodic grid."""
    from paper_0706_0405_amd import vn
    import paper_0706_0405_amd as lb
    from workloads import problems as P

    cfgs, _ = P.batched()
    cases, dts, owner = [], [], []
    for k, c in enumerate(cfgs):
        g = lb.Grid.from_workload(c)
        for st in P.batched_vn_states(c):
            cases.append(vn.case(g, st))
            dts.append([a * g.dx / g.c2 for a in P.VN_ALPHAS])
            owner.append(k)
    kx, ky = P.vn_wave_vectors()
    return cfgs, cases, dts, owner, kx, ky


def bench_vn(dev):
    """GPU von Neumann chooser on the 256 batched Riemann problems: for each problem's
    left, right and two star states, the largest stable alpha = dt c2 / dx among the
    candidates over 64 x 4 wave vectors of its periodic grid, the problem taking the
    minimum over its states; with the strict bound (radius <= 1 + 1e-9) and with the
    growth bound of the workload (a mode may grow 2x over 2000 steps)."""
    import torch
    from paper_0706_0405_amd import vn
    from workloads import problems as P

    cfgs, cases, dts, owner, kxl, kyl = vn_cases()
    kx = torch.tensor(kxl, dtype=torch.float64, device=dev)
    ky = torch.tensor(kyl, dtype=torch.float64, device=dev)
    vn.max_stable_dt(cases, dts, kx, ky, 1e-9)        # warm (module load, first launch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best = vn.max_stable_dt(cases, dts, kx, ky, 1e-9)
    t = time.perf_counter() - t0
    points = len(cases) * len(P.VN_ALPHAS) * kx.numel()
    best_run = vn.max_stable_dt(cases, dts, kx, ky, P.VN_TOL)

    def per_problem(b):
        per = {}
        for k, dt, c in zip(owner, b, cases):
            a = dt * c.c2 / c.dx
            per[k] = min(per.get(k, a), a)
        v = sorted(per.values())
        return per, {"min": v[0], "median": v[len(v) // 2], "max": v[-1], "at_least_0.1": sum(a >= 0.1 for a in v)}
    _, strict = per_problem(best)
    per_run, growth = per_problem(best_run)
    ratio = max(c["dt"] * c["c2"] / c["dx"] / per_run[k] for k, c in enumerate(cfgs))
    return {"problems": len(cfgs), "states_per_problem": 4, "alphas": list(P.VN_ALPHAS), "wave_vectors": kx.numel(),
            "points": points, "ms": t * 1e3, "points_per_s": points / t,
            "chosen_alpha_strict": strict, "tol_run": P.VN_TOL, "chosen_alpha_growth_2x_over_run": growth,
            "workload_alpha_over_chosen_max": ratio}


def bench_configs(dev, max_steps=4000):
    """The paper's small configurations at their own sizes, graph-launched (launch- and
    cache-bound: every one of them fits in the Infinity Cache)."""
    import torch
    import paper_0706_0405_amd as lb
    from workloads import problems as P

    cases = [("Sod 200x4", P.sod(), "f64"), ("1000:1 Riemann 2000x4", P.ratio1000(), "f64"),
             ("1000:1 Riemann 2000x4", P.ratio1000(), "f32"),
             ("Mach-30 Riemann 1200x4", P.mach30(), "f64"),
             ("regular reflection 300x90", P.regular_reflection(), "f32"),
             ("double Mach 960x240", P.double_mach(), "f32")]
    out = []
    s = torch.cuda.Stream(device=dev)
    for name, cfg, prec in cases:
        g = lb.Grid.from_workload(cfg)
        steps = min(int(cfg["steps"]), max_steps)
        steps += steps % 2
        rho, ux, uy, p = fields_to(dev, P.init_fields(cfg))
        with torch.cuda.stream(s):
            fa = lb.init(g, rho, ux, uy, p, prec=prec)
            fb = lb.empty(g, prec, dev)
            lb.run(g, fa, fb, steps, prec=prec, use_graph=True)   # capture + first replay
            times = replays(s, lambda: lb.run(g, fa, fb, steps, prec=prec, use_graph=True), settle_ms=50.0, reps=5)
            ms = median(times)
        out.append({"case": name, "grid": [g.nx, g.ny], "storage": prec, "steps": steps,
                    "ms_per_step": ms / steps, "mlups": g.nx * g.ny * steps / (ms * 1e-3) / 1e6,
                    "replays_rel_range": spread(times)["rel_range"]})
    return out


def bench_adjoint(dev, steps=2000):
    """Gradient of a final-density loss w.r.t. the initial density on the 960 x 240
    double-Mach problem (FP32 storage, FP64 adjoint, sqrt(N) checkpoints) vs the plain forward."""
    import torch
    import paper_0706_0405_amd as lb
    from paper_0706_0405_amd import rollout
    from workloads import problems as P

    cfg = P.double_mach(steps=steps)
    g = lb.Grid.from_workload(cfg)
    rho, ux, uy, p = fields_to(dev, P.init_fields(cfg))
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        R = rollout.Rollout(g, ux, uy, p, steps, prec="f32")
        target = R.forward_density(rho * 1.001).detach()
        fa = lb.init(g, rho, ux, uy, p, prec="f32")
        fb = lb.empty(g, "f32", dev)

        def wall(fn, reps=5):
            """Median host wall time of fn() (ended by a device synchronisation)
            over `reps` calls after one untimed call."""
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return median(ts), ts

        def fwd(spp):
            lb.init(g, rho, ux, uy, p, prec="f32", out=fa)
            lb.run(g, fa, fb, steps, prec="f32", steps_per_pass=spp)

        t_fwd, ts_fwd = wall(lambda: fwd(0))
        t_fwd1, _ = wall(lambda: fwd(1))
        r0 = rho.clone().requires_grad_(True)
        res = {}

        def grad_once():
            res["loss"], res["grad"] = R.loss_and_grad(r0, target)

        t_grad, ts_grad = wall(grad_once)
        grad = res["grad"]
    return {"grid": [g.nx, g.ny], "steps": steps, "checkpoint_every": R.seg, "forward_ms": t_fwd * 1e3,
            "gradient_ms": t_grad * 1e3, "ratio": t_grad / t_fwd,
            "forward_one_step_per_launch_ms": t_fwd1 * 1e3, "ratio_vs_one_step_forward": t_grad / t_fwd1,
            "grad_finite": bool(torch.isfinite(grad).all()),
            "timing": "median host wall time of 5 calls after one untimed call",
            "forward_ms_range": [min(ts_fwd) * 1e3, max(ts_fwd) * 1e3],
            "gradient_ms_range": [min(ts_grad) * 1e3, max(ts_grad) * 1e3]}


def cpu_baseline(target_s=15.0):
    """The FP64 CPU oracle on a bounded sample of the benchmark workload."""
    import torch
    from oracle import scheme
    from workloads import problems as P

    cfg = P.roofline_grid()
    sample = dict(cfg, nx=1024, ny=512)
    pb = scheme.Problem.from_dict(sample)
    f = scheme.init(pb, *P.init_fields(sample))
    t0 = time.perf_counter()
    f = scheme.step(pb, f, 0)
    t1 = time.perf_counter() - t0
    n = max(1, min(200, int(target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    f = scheme.run(pb, f, n, 1)
    dt = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
    except OSError:
        pass
    # the paper's configurations at their own sizes: median time of one step over 20 steps
    configs = []
    for name, c in (("Sod 200x4", P.sod()), ("1000:1 Riemann 2000x4", P.ratio1000()),
                    ("Mach-30 Riemann 1200x4", P.mach30()), ("regular reflection 300x90", P.regular_reflection()),
                    ("double Mach 960x240", P.double_mach())):
        q = scheme.Problem.from_dict(c)
        fc = scheme.init(q, *P.init_fields(c))
        ts = []
        for k in range(20):
            t0 = time.perf_counter()
            fc = scheme.step(q, fc, k)
            ts.append(time.perf_counter() - t0)
        med = sorted(ts)[len(ts) // 2]
        configs.append({"case": name, "grid": [q.nx, q.ny], "ms_per_step": med * 1e3,
                        "mlups": q.nx * q.ny / med / 1e6})
    # the 256 batched problems, 4 steps each, one after the other
    bcfgs, _ = P.batched(nprob=256, seed=0, steps=2000)
    sites = 0
    t0 = time.perf_counter()
    for c in bcfgs:
        q = scheme.Problem.from_dict(c)
        scheme.run(q, scheme.init(q, *P.init_fields(c)), 4, 1)
        sites += q.nx * q.ny
    tb = time.perf_counter() - t0
    # the von Neumann scan: the oracle's amplification-matrix modulus on a sample of the
    # scanner's points (every 97th case, every 37th wave vector, the first candidate step)
    from oracle import vonneumann as ovn
    _, cases, dts, _, kx, ky = vn_cases()
    vsample = [(c, q) for c in range(0, len(cases), 97) for q in range(0, len(kx), 37)]
    t0 = time.perf_counter()
    js = {}
    for c, q in vsample:
        cc = cases[c]
        prm = {"c1": cc.c1, "c2": cc.c2, "eta0": cc.eta0, "gamma": cc.gamma, "tau": cc.tau, "beta": cc.beta,
               "dt": dts[c][0], "dx": cc.dx, "lam": [cc.lam[i] for i in range(9)]}
        stt = (cc.rho, cc.ux, cc.uy, cc.T)
        if c not in js:
            js[c] = ovn.collision_jacobian(*stt, cc.c1, cc.c2, cc.eta0, cc.gamma)
        ovn.max_modulus(stt, prm, kx[q], ky[q], js[c])
    tv = time.perf_counter() - t0
    return {"value": pb.nx * pb.ny * n / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(),
            "kind": "oracle", "host_cpu": model, "host_threads": os.cpu_count(),
            "sample": "FP64 oracle, %d steps of the same double-Mach problem at the same spacing on a "
                      "%dx%d grid (%.1f s)" % (n, pb.nx, pb.ny, dt),
            "configs": configs,
            "batched": {"problems": len(bcfgs), "steps_each": 4, "s": tb, "mlups": sites * 4 / tb / 1e6,
                        "sample": "the 256 batched problems one after the other in this process"},
            "vn_scan": {"points": len(vsample), "s": tv, "points_per_s": len(vsample) / tv,
                        "sample": "every 97th state case, every 37th wave vector, first candidate time step"}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and adjoint measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--prec", choices=["f64", "f32", "both"], default="both")
    ap.add_argument("--profile-run", action="store_true",
                    help="minimal repetition in every leg (for rocprofv3 counter passes); figures not for reporting")
    ap.add_argument("--legs", default="all",
                    help="comma-separated subset of step,batched,adjoint,adjoint_step,vn,configs (for profiling "
                         "one leg; without 'step' the line carries no headline value)")
    args = ap.parse_args()
    global PROFILE
    PROFILE = args.profile_run
    legs = {"step", "batched", "adjoint", "adjoint_step", "vn", "configs"} if args.legs == "all" \
        else set(args.legs.split(","))
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    # a multiple of 12: all two-step passes (their count even) or all three-step
    # passes (an even count), the result in the first buffer either way
    args.steps += (-args.steps) % 12

    import torch
    import paper_0706_0405_amd as lb
    lb._lib.lib()        # fail loudly if the HIP library is missing
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)

    res, one, two = {}, {}, {}
    for prec in (("f64", "f32") if args.prec == "both" else (args.prec,)) if "step" in legs else ():
        # lb_run's default: three steps per pass on FP64 arrays, two on FP32
        spp = 3 if prec == "f64" else 2
        log("timing", prec, "lb_run on the roofline grid, %d steps per pass" % spp)
        res[prec] = time_step(prec, args.steps, args.warmup, dev, per_pass=spp)
        log(prec, json.dumps(res[prec]))
        if prec == "f64":
            log("timing", prec, "lb_run on the roofline grid, two steps per pass")
            two[prec] = time_step(prec, args.steps, args.warmup, dev, per_pass=2)
            log(prec, json.dumps(two[prec]))
        log("timing", prec, "lb_run on the roofline grid, one step per launch")
        one[prec] = time_step(prec, args.steps, args.warmup, dev, per_pass=1)
        log(prec, json.dumps(one[prec]))
    head = "f64" if "f64" in res else "f32"
    copy = None
    if res:
        log("timing a device copy of the same size")
        copy = copy_bandwidth(dev)
        for r_ in list(res.values()) + list(one.values()) + list(two.values()):
            r_["roofline"]["frac_of_device_copy"] = r_["roofline"]["achieved"] / copy["gbs"]
    extras = {}
    if not args.no_extras:
        if "batched" in legs:
            log("timing batched problems")
            extras["batched"] = bench_batched(dev)
            log(json.dumps(extras["batched"]))
        if "adjoint" in legs:
            log("timing adjoint")
            extras["adjoint"] = bench_adjoint(dev)
            log(json.dumps(extras["adjoint"]))
        if "adjoint_step" in legs:
            log("timing one adjoint step on the roofline grid")
            fwd = one["f32"]["ms_per_step"] if "f32" in one else None
            extras["adjoint_step"] = bench_adjoint_step(dev, fwd)
            log(json.dumps(extras["adjoint_step"]))
        if "vn" in legs:
            log("timing the von Neumann chooser")
            extras["vn_scan"] = bench_vn(dev)
            log(json.dumps(extras["vn_scan"]))
        if "configs" in legs:
            log("timing the small configurations at their own sizes")
            extras["configs"] = bench_configs(dev)
            log(json.dumps(extras["configs"]))
    cpu = None
    if not args.no_cpu and res:
        log("timing CPU oracle sample")
        cpu = cpu_baseline()
    if not res:   # a partial run (profiling one leg): no headline
        print(json.dumps({"partial_run": sorted(legs), **extras}), flush=True)
        return
    r = res[head]
    line = {
        "metric": "MLUPS vs HBM roofline (fp64/fp32); batched speedup; adjoint/forward ratio",
        "value": r["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "double-Mach-reflection field, %dx%d grid, %s storage, FDLB steps through lb_run "
                               "(%d time steps per pass)" % (r["grid"][0], r["grid"][1], head.upper(),
                                                             r["steps_per_pass"]),
                   "storage": head, "steps_per_pass": r["steps_per_pass"]},
        "roofline": r["roofline"],
        "replays": r["replays"],
        "mlups_vs_one_step_hbm_bound": r["mlups_vs_one_step_hbm_bound"],
        "one_step_per_launch": {p: {"value": one[p]["mlups"], "unit": "MLUPS", "ms_per_step": one[p]["ms_per_step"],
                                    "roofline": one[p]["roofline"]} for p in one},
        "cpu_baseline": cpu,
        "device_copy": copy,
    }
    if "f64" in two:
        line["fp64_two_steps_per_pass"] = {"value": two["f64"]["mlups"], "unit": "MLUPS",
                                           "ms_per_step": two["f64"]["ms_per_step"], "steps_per_pass": 2,
                                           "replays": two["f64"]["replays"], "roofline": two["f64"]["roofline"]}
    if "f32" in res and head != "f32":
        line["fp32_storage"] = {"value": res["f32"]["mlups"], "unit": "MLUPS", "ms_per_step": res["f32"]["ms_per_step"],
                                "dtype": "f64 arithmetic, f32 storage", "steps_per_pass": 2,
                                "mlups_vs_one_step_hbm_bound": res["f32"]["mlups_vs_one_step_hbm_bound"],
                                "replays": res["f32"]["replays"],
                                "roofline": res["f32"]["roofline"]}
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
