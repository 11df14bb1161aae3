"""GPU adjoint: lb_step_adjoint / lb_init_adjoint and the checkpointed rollout
gradient against the oracle's autograd tape and central finite differences."""
import numpy as np
import pytest
import torch

from oracle import scheme
from workloads import problems as P

from tests._util import F64, say
from tests.test_gpu_parity import BC_SETS, _smooth_cfg

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _lb():
    import paper_0706_0405_amd as lb
    return lb


def _put(lb, g, arr, prec="f64"):
    buf = lb.empty(g, prec, DEV)
    buf.zero_()
    buf[:, :, :g.nx] = torch.as_tensor(arr).to(buf.dtype).to(DEV)
    return buf


@pytest.mark.parametrize("bcs", ["periodic", "walls", "outflow", "inflow", "mixed_split", "walls_split",
                                 "xperiodic"])
@pytest.mark.parametrize("size", [(37, 11), (1, 4), (70, 1)], ids=lambda s: "%dx%d" % s)
def test_step_adjoint_matches_oracle_vjp(bcs, size):
    """One step's vector-Jacobian product against autograd through the oracle step."""
    lb = _lb()
    nx, ny = size
    cfg = _smooth_cfg(nx, ny, BC_SETS[bcs], tau=1.3)
    say("case adjoint", bcs, nx, ny)
    g = lb.Grid.from_workload(cfg)
    pb = scheme.Problem.from_dict(cfg)
    f0 = torch.tensor(P.random_distributions(nx, ny, seed=31), dtype=F64)
    w = torch.tensor(np.random.default_rng(32).standard_normal((9, ny, nx)), dtype=F64)
    n = 7
    _, vjp = torch.autograd.functional.vjp(lambda f: scheme.step(pb, f, n), f0, w)
    got = lb.step_adjoint(g, _put(lb, g, f0), _put(lb, g, w), n=n)
    got = got[:, :, :nx].cpu()
    err = float((got - vjp).abs().max() / vjp.abs().max())
    say("vjp err", err)
    assert err < 1e-13


def test_roofline_grid_adjoint_sampled_rows():
    """One adjoint step on the 8192 x 2048 benchmark grid, as the benchmark launches it
    (default tiles), in both storage precisions of f. g^{n+1} is nonzero only on the
    rows next to the sampled ones, so the sampled rows of g^n are exact; against
    autograd through the oracle's step of those rows (f as stored)."""
    lb = _lb()
    cfg = P.roofline_grid()
    g = lb.Grid.from_workload(cfg)
    pb = scheme.Problem.from_dict(cfg)
    rows = [0, 1, 31, 32, 1023, 1024, 2047]
    win = sorted({min(max(r + d, 0), g.ny - 1) for r in rows for d in (-1, 0, 1)})
    raw = P.random_distributions(g.nx, g.ny, seed=41)
    wt = torch.tensor(np.random.default_rng(42).standard_normal((9, len(win), g.nx)), dtype=F64)
    G = torch.zeros(9, g.ny, g.nx, dtype=F64)
    G[:, win] = wt
    for prec in ("f64", "f32"):
        say("case roofline adjoint", prec)
        f0 = torch.tensor(raw, dtype=torch.float64 if prec == "f64" else torch.float32).to(F64)
        f = f0.clone().requires_grad_(True)
        (scheme.step_rows(pb, f, 5, win) * wt).sum().backward()
        want = f.grad[:, rows]
        got = lb.step_adjoint(g, _put(lb, g, f0, prec), _put(lb, g, G), n=5, prec=prec)
        got = got[:, rows, :g.nx].cpu()
        torch.cuda.empty_cache()
        err = float((got - want).abs().max() / want.abs().max())
        say("roofline adjoint", prec, "err", err)
        assert err < 1e-13


def test_init_adjoint_matches_oracle():
    lb = _lb()
    cfg = P.double_mach(nx=48, ny=12)
    g = lb.Grid.from_workload(cfg)
    pb = scheme.Problem.from_dict(cfg)
    r, u, v, p = [torch.tensor(a, dtype=F64) for a in P.init_fields(cfg)]
    w = torch.tensor(np.random.default_rng(3).standard_normal((9, 12, 48)), dtype=F64)
    _, want = torch.autograd.functional.vjp(lambda rr: scheme.init(pb, rr, u, v, p), r, w)
    got = lb.init_adjoint(g, *[t.to(DEV).contiguous() for t in (r, u, v, p)], _put(lb, g, w)).cpu()
    assert float((got - want).abs().max() / want.abs().max()) < 1e-14


def test_adjoint_dot_product_with_finite_differences():
    """<(S(f + e v) - S(f - e v)) / 2e, w> = <v, S^T w> on the GPU FP64 step."""
    lb = _lb()
    cfg = P.double_mach(nx=120, ny=40)
    g = lb.Grid.from_workload(cfg)
    rng = np.random.default_rng(5)
    f0 = torch.tensor(P.random_distributions(g.nx, g.ny, seed=6), dtype=F64)
    v = torch.tensor(rng.standard_normal(f0.shape), dtype=F64)
    w = torch.tensor(rng.standard_normal(f0.shape), dtype=F64)
    eps = 1e-6
    outs = []
    for sgn in (1.0, -1.0):
        fa = _put(lb, g, f0 + sgn * eps * v)
        fb = lb.empty(g, "f64", DEV)
        lb.step(g, fa, fb, 3)
        outs.append(fb[:, :, :g.nx].cpu())
    jv = (outs[0] - outs[1]) / (2 * eps)
    jtw = lb.step_adjoint(g, _put(lb, g, f0), _put(lb, g, w), n=3)[:, :, :g.nx].cpu()
    lhs = float((jv * w).sum())
    rhs = float((v * jtw).sum())
    say("dot", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)


def _dmr_problem(nx, ny, steps):
    cfg = P.double_mach(nx=nx, ny=ny, steps=steps)
    fields = P.init_fields(cfg)
    target = P.dmr_target_density(cfg, fields[0])
    return cfg, fields, target


def _gpu_gradient(cfg, fields, target_rho, prec, seg=None, keep_all=False):
    lb = _lb()
    from paper_0706_0405_amd import rollout
    g = lb.Grid.from_workload(cfg)
    rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in fields]
    R = rollout.Rollout(g, ux, uy, p, cfg["steps"], prec=prec, seg=seg, keep_all=keep_all)
    tgt = R.forward_density(torch.tensor(target_rho, dtype=F64, device=DEV))
    loss, grad = R.loss_and_grad(rho, tgt)
    return R, loss, grad, tgt


def test_rollout_gradient_matches_oracle_tape():
    """The 48 x 12 double-Mach problem: GPU FP64 rollout gradient (sqrt(N) checkpoints)
    against reverse-mode autograd through the oracle (init, N steps, density, loss)."""
    steps = 60
    cfg, fields, target = _dmr_problem(48, 12, steps)
    R, loss, grad, tgt = _gpu_gradient(cfg, fields, target, "f64")
    pb = scheme.Problem.from_dict(cfg)
    r0 = torch.tensor(fields[0], dtype=F64, requires_grad=True)
    u, v, p = [torch.tensor(a, dtype=F64) for a in fields[1:]]
    f = scheme.run(pb, scheme.init(pb, r0, u, v, p), steps)
    rho = scheme.fields(pb, f)[0]
    L = ((rho - tgt.cpu()) ** 2).sum()
    L.backward()
    want = r0.grad
    err = float((grad.cpu() - want).abs().max() / want.abs().max())
    say("tape err", err, "loss", float(loss), float(L.detach()))
    assert abs(float(loss) - float(L.detach())) <= 1e-10 * float(L.detach())
    assert err < 1e-10


def test_checkpoint_interval_does_not_change_the_gradient():
    cfg, fields, target = _dmr_problem(64, 16, 50)
    grads = [_gpu_gradient(cfg, fields, target, "f64", seg=s)[2] for s in (1, 7, 50)]
    assert torch.equal(grads[0], grads[1]) and torch.equal(grads[0], grads[2])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_keeping_every_state_gives_the_same_gradient(prec):
    """keep_all: every state recorded during the forward (two steps per pass), no
    recomputation; bitwise the gradient of the checkpointed sweep, odd step count."""
    cfg, fields, target = _dmr_problem(64, 16, 51)
    ref = _gpu_gradient(cfg, fields, target, prec, seg=7)[2]
    got = _gpu_gradient(cfg, fields, target, prec, keep_all=True)[2]
    assert torch.isfinite(ref).all()
    assert torch.equal(got, ref)


def _oracle_tape_gradient(cfg, fields, tgt, steps, storage=None):
    """Reverse-mode autograd through the oracle (init, steps, density, loss); with
    storage=float32 every stored state is rounded to float32 on the way forward and
    the rounding is the identity on the way back (as the library's adjoint treats it)."""
    pb = scheme.Problem.from_dict(cfg)
    r0 = torch.tensor(fields[0], dtype=F64, requires_grad=True)
    u, v, p = [torch.tensor(a, dtype=F64) for a in fields[1:]]

    def st(f):
        return f if storage is None else f + (scheme.store(f.detach(), storage) - f.detach())

    f = st(scheme.init(pb, r0, u, v, p))
    for n in range(steps):
        f = st(scheme.step(pb, f, n))
    rho = scheme.fields(pb, f)[0]
    L = ((rho - tgt) ** 2).sum()
    L.backward()
    return float(L.detach()), r0.grad


def test_fp32_storage_rollout_gradient_matches_oracle_tape():
    """The 48 x 12 double-Mach problem in FP32 storage: the GPU gradient (FP32 f, FP64
    adjoint, sqrt(N) checkpoints) against the oracle's tape of the same FP32-storage
    forward, element by element within 1e-10 of the largest component."""
    steps = 60
    cfg, fields, target = _dmr_problem(48, 12, steps)
    R, loss, grad, tgt = _gpu_gradient(cfg, fields, target, "f32")
    L, want = _oracle_tape_gradient(cfg, fields, tgt.cpu(), steps, storage=torch.float32)
    err = float((grad.cpu() - want).abs().max() / want.abs().max())
    say("fp32 tape err", err, "loss", float(loss), L)
    assert abs(float(loss) - L) <= 1e-10 * L
    assert err < 1e-10


def test_rollout_gradient_central_differences_on_full_grid():
    """960 x 240 double-Mach problem, 2000 steps, FP64: the adjoint gradient g against
    central differences d(eps) at every cell of the 48 x 12 crop at the wall start (576
    cells, central differences at eps = 1e-4 rho and eps/2: 2304 forward runs). The
    error of d(eps) is truncation (O(eps^2), about 4/3 of d(eps) - d(eps/2)) plus the
    rounding noise of the loss difference (about 1e-6 of g here: the two perturbed
    2000-step trajectories round differently), which d(eps) - d(eps/2) also measures.
    Bar per cell: |d(eps) - g| <= 1e-6 max(|g|, 1e-3 max|g|) + 2 |d(eps) - d(eps/2)|."""
    lb = _lb()
    cfg, fields, target = _dmr_problem(960, 240, 2000)
    R, loss, grad, tgt = _gpu_gradient(cfg, fields, target, "f64")
    g = R.g
    rho, ux, uy, p = [torch.tensor(np.ascontiguousarray(a), dtype=F64, device=DEV) for a in fields]
    x0 = int(round(cfg["x0"] / cfg["dx"]))
    fa = lb.empty(g, "f64", DEV)
    fb = lb.empty(g, "f64", DEV)

    def loss_at(r):
        lb.init(g, r, ux, uy, p, out=fa)
        out = lb.run(g, fa, fb, cfg["steps"], use_graph=True)
        rN = lb.moments(g, out, flags=False)[0]
        return float(((rN - tgt) ** 2).sum())

    scale = float(grad.abs().max())
    grad_c = grad.cpu()
    rp = rho.clone()

    def central(y, x, eps):
        rp[y, x] = rho[y, x] + eps
        lp = loss_at(rp)
        rp[y, x] = rho[y, x] - eps
        lm = loss_at(rp)
        rp[y, x] = rho[y, x]
        return (lp - lm) / (2 * eps)

    worst, worst_rel, spread_used, bad = 0.0, 0.0, 0, []
    for y in range(12):
        for x in range(x0, x0 + 48):
            eps = 1e-4 * float(rho[y, x])
            d1 = central(y, x, eps)
            d2 = central(y, x, 0.5 * eps)
            ad = float(grad_c[y, x])
            base = 1e-6 * max(abs(ad), 1e-3 * scale)
            tol = base + 2.0 * abs(d1 - d2)
            worst = max(worst, abs(d1 - ad) / tol)
            worst_rel = max(worst_rel, abs(d1 - ad) / max(abs(ad), 1e-3 * scale))
            spread_used += int(abs(d1 - ad) > base)
            if abs(d1 - ad) > tol:
                bad.append((y, x, d1, d2, ad))
    say("central differences over 576 cells: worst |d - g| / bar", worst, "worst relative |d - g|", worst_rel,
        "cells beyond 1e-6 relative (within the step-size spread):", spread_used, "failing", len(bad), bad[:5])
    assert not bad


def test_fp32_storage_gradient_close_to_fp64():
    """The 960 x 240 double-Mach gradient (2000 steps) in FP32 storage against FP64
    storage, element by element: |g32 - g64| <= 2e-3 max|g64| at every cell and
    relative L2 <= 1e-3 (FP32 rounding of the 2000 stored states perturbs the
    trajectory the adjoint runs along)."""
    cfg, fields, target = _dmr_problem(960, 240, 2000)
    _, _, g64, tgt = _gpu_gradient(cfg, fields, target, "f64")
    _, _, g32, _ = _gpu_gradient(cfg, fields, target, "f32")
    scale = float(g64.abs().max())
    d = (g32 - g64).abs()
    rel = float((g32 - g64).norm() / g64.norm())
    big = g64.abs() > 0.1 * scale
    say("fp32 vs fp64 gradient: rel L2", rel, "max |diff| / max|g64|", float(d.max()) / scale,
        "max relative diff where |g64| > 0.1 max", float((d[big] / g64.abs()[big]).max()),
        "cells above 1e-3 max:", int((d > 1e-3 * scale).sum()))
    assert float(d.max()) <= 2e-3 * scale
    assert rel < 1e-3
