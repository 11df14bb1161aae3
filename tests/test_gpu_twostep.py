"""Two steps per pass (lb_run's temporal blocking) against one step per launch.

The two-step kernel keeps the intermediate state in registers, rounded as a stored
step rounds it, and forms its ghosts as the one-step kernel forms them from the
stored state, so lb_run must give bitwise the same array either way: on every
boundary set, on ragged sizes around the 62-column wavefront strips, for every
launch shape, odd and even step counts, and time-dependent (shock) edges."""
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


def _pair(lb, cfg, prec, nsteps, n0=0, tile=None, graph=False, src=None):
    """(one step per launch, two steps per pass) results of lb_run from the same input."""
    g = lb.Grid.from_workload(cfg)
    if src is None:
        rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]
        f0 = lb.init(g, rho, ux, uy, p, prec=prec)
    else:
        f0 = lb.empty(g, prec, DEV)
        f0.zero_()
        f0[:, :, :g.nx] = src.to(f0.dtype).to(DEV)
    res = []
    for spp in (1, 2):
        fa, fb = f0.clone(), lb.empty(g, prec, DEV)
        out = lb.run(g, fa, fb, nsteps, n0=n0, prec=prec, tile=tile, use_graph=graph, steps_per_pass=spp)
        res.append(lb.interior(g, out).clone())
    return res


def _same(a, b):
    eq = (a == b) | (torch.isnan(a) & torch.isnan(b))
    return bool(eq.all())


SIZES = [(77, 13), (64, 3), (3, 2), (62, 7), (63, 9), (124, 5), (125, 33), (200, 70), (1, 5), (130, 1)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bcs", list(BC_SETS))
@pytest.mark.parametrize("size", SIZES, ids=lambda s: "%dx%d" % s)
def test_two_steps_per_pass_bitwise_equal(bcs, size, prec):
    lb = _lb()
    nx, ny = size
    cfg = _smooth_cfg(nx, ny, BC_SETS[bcs])
    say("case two-step", bcs, nx, ny, prec)
    one, two = _pair(lb, cfg, prec, 8, n0=3)
    assert torch.isfinite(one).all()
    assert _same(one, two)


@pytest.mark.parametrize("nsteps", [1, 2, 3, 4, 5, 6, 7, 9, 12])
def test_step_counts_and_result_buffer(nsteps):
    lb = _lb()
    cfg = _smooth_cfg(90, 20, BC_SETS["mixed_split"])
    one, two = _pair(lb, cfg, "f64", nsteps, n0=1)
    assert _same(one, two)


@pytest.mark.parametrize("tile", [(64, 1), (64, 2), (128, 3), (256, 5), (256, 32), (128, 7, 8), (64, 4, 16),
                                  (256, 64)], ids=str)
def test_every_launch_shape(tile):
    lb = _lb()
    cfg = _smooth_cfg(300, 45, BC_SETS["walls_split"])
    for prec in ("f64", "f32"):
        one, two = _pair(lb, cfg, prec, 6, tile=tile)
        assert _same(one, two)


def test_double_mach_shock_edge_and_graph():
    """Time-dependent shock ghosts on the top edge (the second step of a pass uses
    time index n+1), graph-captured, from an odd start index."""
    lb = _lb()
    cfg = P.double_mach(nx=240, ny=60, alpha=0.0125)
    for prec in ("f64", "f32"):
        one, two = _pair(lb, cfg, prec, 40, n0=7, graph=True)
        say("dmr", prec, "equal", _same(one, two))
        assert _same(one, two)


def test_random_non_equilibrium_input_fp32():
    """Random distributions (far from equilibrium) in float storage: the
    intermediate state's rounding to float must match a stored step."""
    lb = _lb()
    cfg = _smooth_cfg(150, 40, BC_SETS["inflow"])
    src = torch.tensor(P.random_distributions(150, 40, seed=17), dtype=F64)
    one, two = _pair(lb, cfg, "f32", 4, src=src)
    assert _same(one, two)
