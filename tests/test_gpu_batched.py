"""GPU batched step: many independent problems of uneven length in one packed
array, advanced by one graph launch; bitwise equal to single-problem runs and
within the FP32-storage bound of the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import scheme
from workloads import problems as P

from tests._util import F64, gpu_run, rel_l1, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _lb():
    import paper_0706_0405_amd as lb
    return lb


def _fields(cfg):
    return [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]


def _bits(t):
    """Bit pattern of a float tensor (NaN payloads included) for exact comparison."""
    t = t.contiguous()
    return t.view(torch.int32 if t.dtype == torch.float32 else torch.int64)


def _make(cfgs, prec="f32"):
    lb = _lb()
    grids = [lb.Grid.from_workload(c) for c in cfgs]
    s = torch.cuda.Stream()
    B = lb.Batch(grids, prec)
    fa, fb = B.empty(DEV), B.empty(DEV)
    fa.zero_()
    fb.zero_()
    for k, c in enumerate(cfgs):
        lb.init(grids[k], *_fields(c), prec=prec, out=B.view(fa, k))
    torch.cuda.synchronize()
    return lb, grids, B, fa, fb, s


def test_layout_is_aligned_and_packed():
    cfgs, _ = P.batched(nprob=40, seed=1, steps=10)
    lb, grids, B, fa, fb, s = _make(cfgs)
    prev_end = 0
    for k, g in enumerate(grids):
        assert B.offsets[k] % 64 == 0 and B.pitches[k] % 64 == 0 and B.pitches[k] >= g.nx
        assert B.offsets[k] == prev_end
        prev_end = B.offsets[k] + 9 * g.ny * B.pitches[k]
    assert B.total == prev_end


@pytest.mark.parametrize("spp", [1, 2])
@pytest.mark.parametrize("block_x", [64, 128, 256])
def test_batched_equals_single_runs_bitwise(block_x, spp):
    """One or two steps per pass over the packed array; the reference is each problem
    run alone, one step per launch."""
    cfgs, _ = P.batched(nprob=48, seed=2, steps=200)
    lb, grids, B, fa, fb, s = _make(cfgs)
    B.set_tile(block_x, spp)
    with torch.cuda.stream(s):
        out = B.step(fa, fb, 200)
    torch.cuda.synchronize()
    say("case batched tile", block_x, "steps per pass", spp)
    for k, (c, g) in enumerate(zip(cfgs, grids)):
        f1 = lb.init(g, *_fields(c), prec="f32")
        f2 = lb.empty(g, "f32", DEV)
        r = lb.run(g, f1, f2, 200, prec="f32", steps_per_pass=1)
        assert torch.equal(_bits(r[:, :, :g.nx]), _bits(B.view(out, k)[:, :, :g.nx])), k


@pytest.mark.parametrize("nsteps", [1, 3, 6, 7])
def test_batched_step_counts_two_steps_per_pass(nsteps):
    """Odd and even step counts (0-3 single steps before the two-step passes), both
    precisions, without a graph (NULL stream) and with one."""
    cfgs, _ = P.batched(nprob=10, seed=5, steps=nsteps)
    for prec, graph in (("f32", True), ("f64", True), ("f32", False)):
        lb, grids, B, fa, fb, s = _make(cfgs, prec)
        ref_a = fa.clone()
        if graph:
            with torch.cuda.stream(s):
                out = B.step(fa, fb, nsteps)
        else:   # the default stream: launches without a graph
            out = B.step(fa, fb, nsteps)
        torch.cuda.synchronize()
        for k, g in enumerate(grids):
            f1 = B.view(ref_a, k).clone()
            r = lb.run(g, f1, torch.empty_like(f1), nsteps, prec=prec, steps_per_pass=1)
            assert torch.equal(_bits(r[:, :, :g.nx]), _bits(B.view(out, k)[:, :, :g.nx])), (prec, k)


def test_graph_replays_continue_the_run():
    cfgs, _ = P.batched(nprob=16, seed=3, steps=100)
    lb, grids, B, fa, fb, s = _make(cfgs)
    ref_a = fa.clone()
    with torch.cuda.stream(s):
        B.step(fa, fb, 100)
        out = B.step(fa, fb, 100)
    torch.cuda.synchronize()
    for k, g in enumerate(grids):
        f1 = B.view(ref_a, k).clone()
        f2 = torch.empty_like(f1)
        r = lb.run(g, f1, f2, 200, prec="f32")
        assert torch.equal(_bits(r[:, :, :g.nx]), _bits(B.view(out, k)[:, :, :g.nx])), k


def test_batched_against_oracle_fp32_bound():
    """The shortest problems of the 256-problem draw, two of the fast subset and the
    longest, 2000 steps, against the FP64 oracle (rows of a y-uniform problem are
    identical, so the oracle runs one row)."""
    cfgs, rej = P.batched(nprob=256, seed=0, steps=2000)
    order = sorted(range(len(cfgs)), key=lambda k: cfgs[k]["nx"])
    pick = order[:4] + [k for k in range(7, 256, 8) if cfgs[k]["nx"] < 400][:2]   # include the fast subset
    pick.append(order[-1])   # and the longest problem (many interior strips)
    sub = [cfgs[k] for k in pick]
    lb, grids, B, fa, fb, s = _make(sub)
    with torch.cuda.stream(s):
        out = B.step(fa, fb, 2000)
    torch.cuda.synchronize()
    for k, (c, g) in enumerate(zip(sub, grids)):
        r, ux, uy, T, fl = lb.moments(g, B.view(out, k), prec="f32")
        c1 = dict(c, ny=1)
        pb = scheme.Problem.from_dict(c1)
        fo = scheme.run(pb, scheme.init(pb, *P.init_fields(c1)), 2000)
        R = scheme.fields(pb, fo)[0]
        if not (torch.isfinite(R).all() and (R > 0).all() and float(R.max()) < 1e6):
            say("oracle run leaves the physical range for problem", pick[k], "- not compared")
            continue
        e = rel_l1(r[0], R[0])
        say("problem", pick[k], "L", c["nx"], "fast", c["fast"], "rel L1", e)
        assert e < 1e-5


def test_autotuners_pick_valid_shapes_and_keep_results(tmp_path, monkeypatch):
    """lb_autotune (single grid) and the batched block-width tuner return valid launch
    shapes, cache them, and the tuned shapes give the same bits as the defaults."""
    import paper_0706_0405_amd as lb
    from paper_0706_0405_amd import tuning
    monkeypatch.setattr(tuning, "CACHE", str(tmp_path / "tune.json"))
    cfg = P.double_mach(nx=333, ny=77)
    g, f0 = gpu_run(cfg, 0, "f32")
    fa, fb = f0.clone(), torch.empty_like(f0)
    tile = tuning.tile_for(g, fa, fb, prec="f32", reps=2)
    say("tuned tile", tile)
    assert tile[0] in (64, 128, 256) and tile[1] >= 1 and tile[3] in (1, 2)
    assert tuning.tile_for(g, fa, fb, prec="f32") == tile          # from the cache
    _, ref = gpu_run(cfg, 10, "f32")
    _, got = gpu_run(cfg, 10, "f32", tile=tile)
    assert torch.equal(_bits(got[:, :, :g.nx]), _bits(ref[:, :, :g.nx]))
    cfgs, _ = P.batched(nprob=12, steps=10, screen=False)
    grids = [lb.Grid.from_workload(c) for c in cfgs]
    B = lb.Batch(grids, "f32")
    try:
        a, b = B.empty(), B.empty()
        a.zero_()
        b.zero_()
        bx = tuning.batch_block_for(B, a, b, steps=4)
        say("tuned batch block", bx)
        assert bx in (64, 128, 256)
    finally:
        B.close()


def _ref_runs(lb, grids, B, src, nsteps, prec):
    """Each problem run alone from the same input, one step per launch."""
    out = []
    for k, g in enumerate(grids):
        f1 = B.view(src, k).clone()
        out.append(lb.run(g, f1, torch.empty_like(f1), nsteps, prec=prec, steps_per_pass=1).clone())
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_four_row_periodic_batches_every_x_edge(prec):
    """Batches whose problems all have 4 rows and a periodic y axis take a kernel of
    their own (the four rows of a strip in registers); x edges of every kind but
    the moving shock, split edges, ragged widths around the 60-column strips, odd
    and even step counts: bitwise equal to each problem run alone."""
    from tests.test_gpu_parity import _edge, _smooth_cfg
    per = _edge("periodic")
    xedges = [(_edge("outflow"), _edge("outflow")), (_edge("wall", split=2), _edge("inflow")),
              (per, per), (_edge("inflow"), _edge("wall")), (_edge("outflow", split=1), _edge("wall", split=3))]
    widths = [61, 3, 130, 250, 62, 8, 121, 1]
    cfgs = [_smooth_cfg(nx, 4, [*xedges[k % len(xedges)], per, per], seed=k) for k, nx in enumerate(widths)]
    for nsteps in (5, 6):
        lb, grids, B, fa, fb, s = _make(cfgs, prec)
        src = fa.clone()
        with torch.cuda.stream(s):
            out = B.step(fa, fb, nsteps)
        torch.cuda.synchronize()
        ref = _ref_runs(lb, grids, B, src, nsteps, prec)
        for k, g in enumerate(grids):
            assert torch.isfinite(ref[k][:, :, :g.nx]).all()
            assert torch.equal(_bits(ref[k][:, :, :g.nx]), _bits(B.view(out, k)[:, :, :g.nx])), (nsteps, k)
        B.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_mixed_batch_takes_the_general_march(prec):
    """One problem that is not 4 rows with a periodic y axis sends the whole batch
    through the general two-step march; still bitwise equal to single runs."""
    from tests.test_gpu_parity import BC_SETS, _edge, _smooth_cfg
    per = _edge("periodic")
    cfgs = [_smooth_cfg(90, 4, [_edge("outflow"), _edge("outflow"), per, per], seed=1),
            _smooth_cfg(77, 13, BC_SETS["walls"], seed=2),
            _smooth_cfg(64, 4, BC_SETS["walls_split"], seed=3),
            _smooth_cfg(125, 7, BC_SETS["inflow"], seed=4),
            _smooth_cfg(30, 2, BC_SETS["periodic"], seed=5)]
    lb, grids, B, fa, fb, s = _make(cfgs, prec)
    src = fa.clone()
    with torch.cuda.stream(s):
        out = B.step(fa, fb, 7)
    torch.cuda.synchronize()
    ref = _ref_runs(lb, grids, B, src, 7, prec)
    for k, g in enumerate(grids):
        assert torch.equal(_bits(ref[k][:, :, :g.nx]), _bits(B.view(out, k)[:, :, :g.nx])), k
    B.close()
