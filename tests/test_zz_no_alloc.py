"""lb_invariants_noalloc (the library's fixed per-device array instead of a
workspace) against lb_invariants through the C ABI: bitwise the same totals, on
two calls in a row, the second on a smaller grid, in both storage precisions."""
import ctypes

import numpy as np
import pytest
import torch

from workloads import problems as P

from tests._util import F64, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _field(lb, cfg, prec, seed):
    """A distribution array holding seeded positive values (interior and padding)."""
    g = lb.Grid.from_workload(cfg)
    f = lb.empty(g, prec, DEV)
    rng = np.random.default_rng(seed)
    f.copy_(torch.tensor(rng.uniform(0.5, 1.5, size=tuple(f.shape)), dtype=f.dtype))
    return g, f


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_invariants_equal_the_allocating_entry_point(prec):
    import paper_0706_0405_amd as lb
    from paper_0706_0405_amd import _lib
    L = _lib.lib()
    s = torch.cuda.Stream()
    # the second call on a smaller grid: fewer partial records than the first left behind
    for k, cfg in enumerate((P.double_mach(nx=2000, ny=3000), P.regular_reflection())):
        g, f = _field(lb, cfg, prec, seed=7 + k)
        gc = g.c()
        want = torch.full((4,), float("nan"), dtype=F64, device=DEV)
        got = torch.full((4,), float("nan"), dtype=F64, device=DEV)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            st = ctypes.c_void_p(s.cuda_stream)
            _lib.check(L.lb_invariants(ctypes.byref(gc), _lib.LB_F64 if prec == "f64" else _lib.LB_F32,
                                       ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(want.data_ptr()), st))
            _lib.check(L.lb_invariants_noalloc(ctypes.byref(gc), _lib.LB_F64 if prec == "f64" else _lib.LB_F32,
                                               ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(got.data_ptr()), st))
        torch.cuda.synchronize()
        say("case noalloc", prec, g.nx, g.ny, "totals", got.cpu().tolist())
        assert torch.isfinite(want).all()
        assert torch.equal(got.view(torch.int64), want.view(torch.int64)), (got, want)
        # the totals themselves: mass is the sum of every plane over the interior
        mass = float(f[:, :, :g.nx].to(F64).sum())
        assert abs(float(got[0]) - mass) <= 1e-12 * mass


def test_noalloc_invariants_reject_bad_arguments_before_any_launch():
    from paper_0706_0405_amd import _lib
    import paper_0706_0405_amd as lb
    L = _lib.lib()
    g = lb.Grid.from_workload(P.sod()).c()
    assert L.lb_invariants_noalloc(ctypes.byref(g), 0, None, None, None) == -1
    assert L.lb_invariants_noalloc(ctypes.byref(g), 0, ctypes.c_void_p(1 << 20), None, None) == -1
    assert b"out4" in L.lb_last_error()
