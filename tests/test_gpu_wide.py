"""Distribution arrays of 4 GiB and more (per-plane resources over each tile's rows).

The large-array kernels differ from the others only in how they address memory, so
on data that repeat every 64 rows of a y-periodic grid they must give every element
bitwise equal to the 64-row grid run by the regular kernels; with non-periodic
edges, sampled rows of one step are checked against the oracle row by row and the
rows along each y edge against a 128-row grid holding the same rows (bitwise)."""
import numpy as np
import pytest
import torch

from oracle import scheme
from workloads import problems as P

from tests._util import F64, say
from tests.test_gpu_parity import _edge

pytestmark = pytest.mark.gpu
DEV = "cuda"
NX = 8192
# rows that take each precision's array past 4 GiB (9 * 8192 * ny * bytes >= 2^32)
NY_WIDE = {"f64": 114 * 64, "f32": 228 * 64}
DT = {"f64": torch.float64, "f32": torch.float32}


def _lb():
    import paper_0706_0405_amd as lb
    return lb


def _grid(lb, ny, edges):
    cfg = P.periodic_smooth(nx=NX, ny=ny)
    cfg["edges"] = edges
    return lb.Grid.from_workload(cfg)


def _block(ny, seed):
    """Seeded random non-equilibrium distributions, (9, ny, NX) float64 on the CPU."""
    return torch.tensor(P.random_distributions(NX, ny, seed=seed), dtype=F64)


def _put(lb, g, prec, src):
    buf = lb.empty(g, prec, DEV)
    buf.zero_()
    buf[:, :, :g.nx] = src.to(DT[prec]).to(DEV)
    return buf


def _is_wide(g, nbytes):
    return 9 * g.pitch * g.ny * nbytes >= 1 << 32


@pytest.mark.parametrize("spp", [1, 2])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_periodic_repeat_bitwise_equal_to_small_grid(prec, spp):
    """4 steps (one or two per pass), then moments, on a y-periodic 8192-wide grid of
    64-row repeats."""
    lb = _lb()
    per = [_edge("periodic") for _ in range(4)]
    small = _grid(lb, 64, per)
    big = _grid(lb, NY_WIDE[prec], per)
    reps = big.ny // 64
    assert _is_wide(big, 8 if prec == "f64" else 4) and not _is_wide(small, 8)
    say("case wide periodic", prec, big.nx, big.ny)
    s0 = _put(lb, small, prec, _block(64, seed=41))
    Fa = lb.empty(big, prec, DEV)
    Fa.view(9, reps, 64, big.pitch)[:] = s0.unsqueeze(1)
    want = lb.run(small, s0, lb.empty(small, prec, DEV), 4, prec=prec, steps_per_pass=spp).clone()
    Fb = lb.empty(big, prec, DEV)
    got = lb.run(big, Fa, Fb, 4, prec=prec, steps_per_pass=spp)
    same = bool((got.view(9, reps, 64, big.pitch)[..., :NX] == want[:, None, :, :NX]).all())
    say("all elements equal:", same)
    assert same
    r, ux, uy, T, flags = lb.moments(big, got, prec=prec)
    R, UX, UY, TT, _ = lb.moments(small, want, prec=prec)
    for a, b in ((r, R), (ux, UX), (uy, UY), (T, TT)):
        assert bool((a.view(reps, 64, NX) == b[None]).all())
    assert int(flags[0]) == 0
    del Fa, Fb, got, r, ux, uy, T
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_edges_one_step_sampled_rows_and_edge_bands(prec):
    """Inflow / outflow x edges, a split wall below, a wall above: one step from
    random distributions; sampled rows (tile boundaries, both edges, the middle)
    against the oracle, and the 64 rows along each y edge bitwise against a
    128-row grid holding the same input rows."""
    lb = _lb()
    edges = [_edge("inflow"), _edge("outflow"), _edge("wall", split=300), _edge("wall")]
    big = _grid(lb, NY_WIDE[prec], edges)
    ny = big.ny
    say("case wide edges", prec, big.nx, ny)
    src = _block(64, seed=43).repeat(1, ny // 64, 1)
    src[:, -256:] = _block(256, seed=44)           # the top band differs from the rest
    f = _put(lb, big, prec, src)
    out = lb.empty(big, prec, DEV)
    lb.step(big, f, out, 0, prec=prec)
    rows = [0, 1, 2, 31, 32, 33, ny // 2 - 1, ny // 2, ny - 33, ny - 32, ny - 2, ny - 1]
    got = out[:, rows, :NX].cpu().to(F64)
    cfg = P.periodic_smooth(nx=NX, ny=ny)
    cfg["edges"] = edges
    want = scheme.step_rows(scheme.Problem.from_dict(cfg), src.to(DT[prec]).to(F64), 0, rows)
    err = float(((got - want).abs() / want.abs().max()).max())
    say("sampled rows max rel err", err)
    assert err < (1e-13 if prec == "f64" else 1.2e-7)
    lo, hi = out[:, :64, :NX].clone(), out[:, -64:, :NX].clone()
    # four steps, two per pass, equal four single steps on the large array
    a, b = f.clone(), lb.empty(big, prec, DEV)
    two = lb.run(big, a, b, 4, prec=prec, steps_per_pass=2)
    c, d = f, out
    one = lb.run(big, c, d, 4, prec=prec, steps_per_pass=1)
    assert bool((two[..., :NX] == one[..., :NX]).all())
    del a, b, c, d, two, one, f, out
    torch.cuda.empty_cache()
    small = _grid(lb, 128, edges)
    for band, part in ((lo, src[:, :128]), (hi, src[:, -128:])):
        fs = _put(lb, small, prec, part)
        os_ = lb.empty(small, prec, DEV)
        lb.step(small, fs, os_, 0, prec=prec)
        ref = os_[:, :64, :NX] if band is lo else os_[:, -64:, :NX]
        assert bool((band == ref).all())


def test_adjoint_periodic_repeat_bitwise_equal_to_small_grid():
    """One adjoint step with double adjoint arrays past 4 GiB (f in float storage)."""
    lb = _lb()
    per = [_edge("periodic") for _ in range(4)]
    small = _grid(lb, 64, per)
    big = _grid(lb, NY_WIDE["f64"], per)
    reps = big.ny // 64
    assert _is_wide(big, 8)
    say("case wide adjoint", big.nx, big.ny)
    f = _block(64, seed=45)
    w = torch.tensor(np.random.default_rng(46).standard_normal((9, 64, NX)), dtype=F64)
    fs, ws = _put(lb, small, "f32", f), _put(lb, small, "f64", w)
    want = lb.step_adjoint(small, fs, ws, n=3, prec="f32")
    Fb = lb.empty(big, "f32", DEV)
    Fb.view(9, reps, 64, big.pitch)[:] = fs.unsqueeze(1)
    Wb = lb.empty(big, "f64", DEV)
    Wb.view(9, reps, 64, big.pitch)[:] = ws.unsqueeze(1)
    got = lb.step_adjoint(big, Fb, Wb, n=3, prec="f32")
    same = bool((got.view(9, reps, 64, big.pitch)[..., :NX] == want[:, None, :, :NX]).all())
    say("all elements equal:", same)
    assert same
    del Fb, Wb, got
    torch.cuda.empty_cache()
