"""lb_run_record (every state of a segment kept, as the checkpointed gradient
recomputes them): two steps per pass with the intermediate state stored on the
way, bitwise equal to one step per launch for every recorded state; buffers that
repeat fall back to single steps and still give the same states."""
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


def _f0(lb, g, cfg, prec):
    rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]
    return lb.init(g, rho, ux, uy, p, prec=prec)


def _single_steps(lb, g, f0, n0, nsteps, prec):
    """States after steps n0 .. n0+nsteps-1, one lb_step per state."""
    out, cur = [], f0
    for j in range(nsteps):
        nxt = lb.empty(g, prec, DEV)
        lb.step(g, cur, nxt, n0 + j, prec=prec)
        out.append(nxt)
        cur = nxt
    return out


def _same(a, b):
    eq = (a == b) | (torch.isnan(a) & torch.isnan(b))
    return bool(eq.all())


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bcs", list(BC_SETS))
@pytest.mark.parametrize("size", [(77, 13), (3, 2), (125, 33), (130, 1)], ids=lambda s: "%dx%d" % s)
def test_recorded_states_bitwise_equal_single_steps(bcs, size, prec):
    lb = _lb()
    nx, ny = size
    cfg = _smooth_cfg(nx, ny, BC_SETS[bcs])
    g = lb.Grid.from_workload(cfg)
    f0 = _f0(lb, g, cfg, prec)
    say("case record", bcs, nx, ny, prec)
    for nsteps in (1, 2, 5, 6):
        ref = _single_steps(lb, g, f0, 3, nsteps, prec)
        outs = [lb.empty(g, prec, DEV) for _ in range(nsteps)]
        lb.api.run_record(g, f0, outs, n0=3, prec=prec)
        torch.cuda.synchronize()
        for j in range(nsteps):
            assert torch.isfinite(lb.interior(g, ref[j])).all()
            assert _same(lb.interior(g, outs[j]), lb.interior(g, ref[j])), (nsteps, j)


def test_moving_shock_edge_odd_start():
    """Double Mach reflection: the top edge's shock ghosts depend on the time index of
    each step, the stored intermediate state included."""
    lb = _lb()
    cfg = P.double_mach(nx=240, ny=60, alpha=0.0125)
    g = lb.Grid.from_workload(cfg)
    for prec in ("f64", "f32"):
        f0 = _f0(lb, g, cfg, prec)
        ref = _single_steps(lb, g, f0, 7, 9, prec)
        outs = [lb.empty(g, prec, DEV) for _ in range(9)]
        lb.api.run_record(g, f0, outs, n0=7, prec=prec)
        torch.cuda.synchronize()
        for j in range(9):
            assert _same(lb.interior(g, outs[j]), lb.interior(g, ref[j])), (prec, j)


def test_repeated_buffers_fall_back_to_single_steps():
    """outs = [A, B, A, B, A]: a two-step pass may not write its input, so the
    library takes single steps where a pass would; the last state is still exact."""
    lb = _lb()
    cfg = _smooth_cfg(90, 20, BC_SETS["mixed_split"])
    g = lb.Grid.from_workload(cfg)
    for prec in ("f64", "f32"):
        f0 = _f0(lb, g, cfg, prec)
        ref = _single_steps(lb, g, f0, 1, 5, prec)
        a, b = lb.empty(g, prec, DEV), lb.empty(g, prec, DEV)
        lb.api.run_record(g, f0, [a, b, a, b, a], n0=1, prec=prec)
        torch.cuda.synchronize()
        assert _same(lb.interior(g, a), lb.interior(g, ref[4]))
        assert _same(lb.interior(g, b), lb.interior(g, ref[3]))
