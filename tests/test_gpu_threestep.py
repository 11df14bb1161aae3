"""Three steps per pass (lb_run's default on FP64 arrays) against one step per launch.

The three-step kernel keeps two intermediate states in registers and forms their
ghosts as the one-step kernel forms them from a stored state, so lb_run must give
bitwise the same array either way: on every boundary set, on ragged sizes around
the 58-column wavefront strips and the 232-column blocks, for every launch shape
(tiles of 1-3 rows put the y-edge march on interior rows too), step counts that
leave single steps before the passes, and time-dependent (shock) edges."""
import numpy as np
import pytest
import torch

from workloads import problems as P

from tests._util import F64, say
from tests.test_gpu_parity import BC_SETS, _smooth_cfg

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _lb():
    import paper_0706_0405_amd as lb
    return lb


def _pair(lb, cfg, nsteps, n0=0, tile=None, graph=False, src=None):
    """(one step per launch, three steps per pass) FP64 results of lb_run from the same input."""
    g = lb.Grid.from_workload(cfg)
    if src is None:
        rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]
        f0 = lb.init(g, rho, ux, uy, p, prec="f64")
    else:
        f0 = lb.empty(g, "f64", DEV)
        f0.zero_()
        f0[:, :, :g.nx] = src.to(DEV)
    res = []
    for spp in (1, 3):
        fa, fb = f0.clone(), lb.empty(g, "f64", DEV)
        out = lb.run(g, fa, fb, nsteps, n0=n0, prec="f64", tile=tile, use_graph=graph, steps_per_pass=spp)
        res.append(lb.interior(g, out).clone())
    return res


def _same(a, b):
    eq = (a == b) | (torch.isnan(a) & torch.isnan(b))
    return bool(eq.all())


SIZES = [(77, 13), (64, 3), (3, 4), (58, 7), (59, 9), (116, 5), (117, 33), (232, 6), (233, 12), (200, 70),
         (1, 5), (130, 3)]


@pytest.mark.parametrize("bcs", list(BC_SETS))
@pytest.mark.parametrize("size", SIZES, ids=lambda s: "%dx%d" % s)
def test_three_steps_per_pass_bitwise_equal(bcs, size):
    lb = _lb()
    nx, ny = size
    cfg = _smooth_cfg(nx, ny, BC_SETS[bcs])
    say("case three-step", bcs, nx, ny)
    one, three = _pair(lb, cfg, 9, n0=3)
    assert torch.isfinite(one).all()
    assert _same(one, three)


@pytest.mark.parametrize("nsteps", [1, 2, 3, 4, 5, 6, 7, 8, 11, 12])
def test_step_counts_and_result_buffer(nsteps):
    lb = _lb()
    cfg = _smooth_cfg(90, 20, BC_SETS["mixed_split"])
    one, three = _pair(lb, cfg, nsteps, n0=1)
    assert _same(one, three)


@pytest.mark.parametrize("tile", [(64, 1), (64, 2), (128, 3), (256, 4), (256, 11), (256, 32), (128, 7, 8),
                                  (64, 4, 16), (256, 64)], ids=str)
@pytest.mark.parametrize("bcs", ["walls_split", "periodic", "xperiodic"])
def test_every_launch_shape(tile, bcs):
    lb = _lb()
    cfg = _smooth_cfg(300, 45, BC_SETS[bcs])
    one, three = _pair(lb, cfg, 6, tile=tile)
    assert _same(one, three)


def test_double_mach_shock_edge_and_graph():
    """Time-dependent shock ghosts on the top edge (the second and third steps of a
    pass use time indices n+1, n+2), graph-captured, from an odd start index."""
    lb = _lb()
    cfg = P.double_mach(nx=240, ny=60, alpha=0.0125)
    for tile in (None, (64, 1), (256, 5)):
        one, three = _pair(lb, cfg, 42, n0=7, graph=True, tile=tile)
        say("dmr", tile, "equal", _same(one, three))
        assert _same(one, three)


def test_random_non_equilibrium_input():
    """Random distributions far from equilibrium through every boundary kind."""
    lb = _lb()
    for bcs in ("inflow", "walls", "mixed_split"):
        cfg = _smooth_cfg(150, 40, BC_SETS[bcs])
        src = torch.tensor(P.random_distributions(150, 40, seed=17), dtype=F64)
        one, three = _pair(lb, cfg, 6, src=src)
        assert _same(one, three)


def test_default_is_three_steps_on_fp64_and_requests_it_cannot_run_are_rejected():
    """steps_per_pass = 0 on an FP64 array of at least 32 rows takes the three-step
    pass (bitwise the explicit request); three steps on FP32 storage or on 2 rows:
    LB_EUNSUPPORTED."""
    from paper_0706_0405_amd import _lib
    lb = _lb()
    cfg = _smooth_cfg(120, 40, BC_SETS["mixed_split"])
    g = lb.Grid.from_workload(cfg)
    rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]
    f0 = lb.init(g, rho, ux, uy, p, prec="f64")
    outs = []
    for spp in (0, 3):
        fa, fb = f0.clone(), lb.empty(g, "f64", DEV)
        outs.append(lb.interior(g, lb.run(g, fa, fb, 9, prec="f64", steps_per_pass=spp)).clone())
    assert _same(outs[0], outs[1])
    f32 = lb.init(g, rho, ux, uy, p, prec="f32")
    with pytest.raises(_lib.LbError) as e:
        lb.run(g, f32, lb.empty(g, "f32", DEV), 3, prec="f32", steps_per_pass=3)
    assert e.value.status == -7
    cfg2 = _smooth_cfg(120, 2, BC_SETS["walls"])
    g2 = lb.Grid.from_workload(cfg2)
    f2 = lb.empty(g2, "f64", DEV)
    f2.fill_(0.1)
    with pytest.raises(_lib.LbError) as e:
        lb.run(g2, f2, lb.empty(g2, "f64", DEV), 3, prec="f64", steps_per_pass=3)
    assert e.value.status == -7
    fa = f2.clone()
    lb.run(g2, fa, lb.empty(g2, "f64", DEV), 3, prec="f64")   # the default falls back to two per pass
