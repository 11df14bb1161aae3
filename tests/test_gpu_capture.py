"""The library under a caller's HIP graph capture: lb_run (launches only, no graph of
its own), lb_moments and lb_invariants_noalloc enqueue nothing but kernels (no
allocation, no memset), so a caller can capture them in its own graph. Each replay,
with the program's own eager work and synchronisations between replays, must equal
the eager result bitwise."""
import numpy as np
import pytest
import torch

from workloads import problems as P

from tests._util import F64, say

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _bits(t):
    t = t.contiguous()
    return t.view(torch.int32 if t.dtype == torch.float32 else torch.int64)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_step_moments_and_noalloc_invariants_replay_under_a_captured_graph(prec):
    import paper_0706_0405_amd as lb
    cfg = P.double_mach(nx=240, ny=60)
    g = lb.Grid.from_workload(cfg)
    fields = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in P.init_fields(cfg)]
    fa = lb.init(g, *fields, prec=prec)
    fb = lb.empty(g, prec, DEV)
    f0 = fa.clone()
    inv = torch.empty(4, dtype=F64, device=DEV)
    # eager reference: 10 steps, then the moments and the totals
    out = lb.run(g, fa, fb, 10, prec=prec)
    want_rho = lb.moments(g, out, prec=prec, flags=False)[0].clone()
    want_inv = lb.invariants(g, out, prec=prec, noalloc=True).clone()
    want_f = lb.interior(g, out).clone()                   # out is fa or fb: replays overwrite it
    torch.cuda.synchronize()
    # the same work captured in a graph of the caller's
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    fa.copy_(f0)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            o = lb.run(g, fa, fb, 10, prec=prec)            # kernels only (use_graph=False)
            rho = lb.moments(g, o, prec=prec, flags=False)[0]
            lb.invariants(g, o, prec=prec, out=inv, noalloc=True)
    for rep in range(3):
        fa.copy_(f0)                                        # eager work between replays
        fb.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say("capture", prec, "replay", rep, "totals", inv.cpu().tolist())
        assert torch.equal(_bits(rho), _bits(want_rho)), rep
        assert torch.equal(_bits(inv), _bits(want_inv)), rep
        assert torch.equal(_bits(lb.interior(g, o)), _bits(want_f)), rep
