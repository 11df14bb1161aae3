"""lb_run's deep pass on 4-row grids with a periodic y axis against one step per launch.

On such grids (the paper's one-dimensional Riemann problems) lb_run's default keeps
the state of a strip on chip (a row per wavefront, the rows exchanged through LDS)
for several steps per pass. Every
intermediate state is rounded to the storage type and its x ghosts are formed as a
single step forms them, so the array must be bitwise the one that one step per
launch gives: for every x-edge kind (split edges too), widths around the strips
of 64 - 2D columns, step counts that leave no, two or more passes plus leftover
single and two-step launches, both storage types, with and without a graph, on
smooth and on random non-equilibrium input, and on the paper's configurations."""
import numpy as np
import pytest
import torch

from workloads import problems as P

from tests._util import F64, say
from tests.test_gpu_parity import _edge, _smooth_cfg

pytestmark = pytest.mark.gpu
DEV = "cuda"

Y = [_edge("periodic"), _edge("periodic")]
X_SETS = {
    "periodic": [_edge("periodic"), _edge("periodic")],
    "walls": [_edge("wall"), _edge("wall")],
    "outflow": [_edge("outflow"), _edge("outflow")],
    "inflow": [_edge("inflow"), _edge("inflow", a=(0.9, -0.4, 0.2, 1.3))],
    "inflow_outflow": [_edge("inflow"), _edge("outflow")],
    "splits": [_edge("wall", split=2), _edge("outflow", split=1)],
    "inflow_split_wall": [_edge("inflow", split=3), _edge("wall")],
}
WIDTHS = [64, 65, 96, 97, 127, 128, 200, 333]


def _lb():
    import paper_0706_0405_amd as lb
    return lb


def _pair(lb, cfg, nsteps, prec, n0=0, graph=False, src=None):
    """(one step per launch, lb_run's default) results from the same input."""
    g = lb.Grid.from_workload(cfg)
    if src is None:
        rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]
        f0 = lb.init(g, rho, ux, uy, p, prec=prec)
    else:
        f0 = lb.empty(g, prec, DEV)
        f0.zero_()
        f0[:, :, :g.nx] = src.to(DEV, f0.dtype)
    res = []
    for spp in (1, 0):
        fa, fb = f0.clone(), lb.empty(g, prec, DEV)
        out = lb.run(g, fa, fb, nsteps, n0=n0, prec=prec, use_graph=graph, steps_per_pass=spp)
        assert (out is fa) == (nsteps % 2 == 0)
        res.append(lb.interior(g, out).clone())
    return res


def _same(a, b):
    eq = (a == b) | (torch.isnan(a) & torch.isnan(b))
    return bool(eq.all())


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("xs", list(X_SETS))
@pytest.mark.parametrize("nx", WIDTHS)
def test_deep_pass_bitwise_equal_to_single_steps(prec, xs, nx):
    lb = _lb()
    cfg = _smooth_cfg(nx, 4, X_SETS[xs] + Y)
    say("case deep single", prec, xs, nx)
    one, deep = _pair(lb, cfg, 37, prec, n0=2)
    assert torch.isfinite(one).all()
    assert _same(one, deep)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("nsteps", [1, 2, 3, 7, 8, 15, 16, 17, 18, 19, 23, 24, 31, 32, 33, 40, 49])
def test_step_counts_and_result_buffer(prec, nsteps):
    lb = _lb()
    cfg = _smooth_cfg(150, 4, X_SETS["inflow_outflow"] + Y)
    one, deep = _pair(lb, cfg, nsteps, prec, n0=1)
    assert _same(one, deep)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("xs", ["outflow", "periodic", "splits"])
def test_graph_replays_and_random_input(prec, xs):
    lb = _lb()
    cfg = _smooth_cfg(211, 4, X_SETS[xs] + Y)
    src = torch.tensor(P.random_distributions(211, 4, seed=17), dtype=F64)
    one, deep = _pair(lb, cfg, 48, prec, graph=True, src=src)
    assert _same(one, deep)
    # a second replay of the cached graph from the same input
    one2, deep2 = _pair(lb, cfg, 48, prec, graph=True, src=src)
    assert _same(deep, deep2) and _same(one, one2)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["sod", "ratio1000", "mach30"])
def test_paper_riemann_configurations(prec, name):
    lb = _lb()
    cfg = getattr(P, name)()
    say("case deep paper config", prec, name, cfg["nx"])
    one, deep = _pair(lb, cfg, 200, prec, graph=True)
    assert torch.isfinite(one).all()
    assert _same(one, deep)


def test_narrow_grids_keep_the_general_passes():
    # below 64 columns lb_run keeps one and two steps per pass: still bitwise
    lb = _lb()
    for nx in (1, 5, 40, 63):
        cfg = _smooth_cfg(nx, 4, X_SETS["walls"] + Y)
        one, other = _pair(lb, cfg, 20, "f64")
        assert _same(one, other)


def test_autotuner_offers_the_deep_pass(tmp_path, monkeypatch):
    """lb_autotune times the sixteen-step pass on such grids too and returns it as
    steps = 0 (lb_run's default there): about three times faster per step than one
    or two steps per launch on the paper's 1000:1 grid; the tuned tile gives the
    same bits."""
    lb = _lb()
    from paper_0706_0405_amd import tuning
    monkeypatch.setattr(tuning, "CACHE", str(tmp_path / "tune.json"))
    cfg = P.ratio1000()
    g = lb.Grid.from_workload(cfg)
    rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]
    f0 = lb.init(g, rho, ux, uy, p, prec="f64")
    tile = tuning.tile_for(g, f0.clone(), lb.empty(g, "f64", DEV), prec="f64", reps=4)
    say("tuned tile 1000:1", tile)
    assert tile[3] == 0 and tile[0] in (64, 128, 256) and tile[1] >= 1
    outs = []
    for kw in ({"steps_per_pass": 1}, {"tile": tile}):
        fa, fb = f0.clone(), lb.empty(g, "f64", DEV)
        outs.append(lb.interior(g, lb.run(g, fa, fb, 70, prec="f64", use_graph=True, **kw)).clone())
    assert _same(outs[0], outs[1])
