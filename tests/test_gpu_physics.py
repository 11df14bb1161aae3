"""GPU runs of the paper's 2D validation problems to their physical end states,
checked against closed-form gas dynamics (properties that hold at any size)."""
import math

import numpy as np
import pytest
import torch

from workloads import gasdyn, problems as P

from tests._util import gpu_fields, gpu_run, say

pytestmark = pytest.mark.gpu


def _patch(field, x, y, dx, half=3):
    i, j = int(round(x / dx - 0.5)), int(round(y / dx - 0.5))
    return float(field[j - half:j + half + 1, i - half:i + half + 1].mean())


def test_regular_reflection_reaches_two_shock_steady_state():
    """Sec. 4.2 regular reflection (Mach 2.9 inflow, 30-degree incident shock, 300 x 90,
    FP32 storage, 20000 steps): the plateaus behind the incident and the reflected shock
    match two-shock theory within 5% in density and pressure, and the field is steady."""
    import paper_0706_0405_amd as lb
    cfg = P.regular_reflection()
    n = cfg["steps"]
    say("case regular reflection", cfg["nx"], cfg["ny"], n)
    g, f = gpu_run(cfg, n, "f32")
    (rho, ux, uy, T), flags = gpu_fields(g, f, "f32")
    assert int(flags[1]) == 0 and int(flags[2]) == 0, flags.tolist()
    fb = lb.empty(g, "f32", f.device)
    fa = f.clone()
    out = lb.run(g, fa, fb, 100, n0=n, prec="f32")
    (rho2, _, _, _), _ = gpu_fields(g, out, "f32")
    resid = float((rho2 - rho).abs().sum() / rho.abs().sum())
    say("steady residual over 100 steps", resid)
    assert resid < 1e-6
    rho, T = rho.cpu().numpy(), T.cpu().numpy()
    p = rho * T
    s2, s3, br = gasdyn.regular_reflection_states(1.4, cfg["inflow"], cfg["wave_angle_deg"])
    dx = cfg["dx"]
    # region 2: above the incident shock, upstream of the reflection point
    r2, p2 = _patch(rho, 1.0, 0.7, dx), _patch(p, 1.0, 0.7, dx)
    # region 3: below the reflected shock, downstream of the reflection point
    theta = -math.degrees(math.atan2(s2[2], s2[1]))
    xw = cfg["ny"] * dx / math.tan(math.radians(cfg["wave_angle_deg"]))
    yr = (2.3 - xw) * math.tan(math.radians(br - theta))
    assert yr > 0.25
    r3, p3 = _patch(rho, 2.3, 0.12, dx), _patch(p, 2.3, 0.12, dx)
    say("region 2 rho %.4f (theory %.4f) p %.4f (%.4f)" % (r2, s2[0], p2, s2[3]))
    say("region 3 rho %.4f (theory %.4f) p %.4f (%.4f)" % (r3, s3[0], p3, s3[3]))
    for got, want in ((r2, s2[0]), (p2, s2[3]), (r3, s3[0]), (p3, s3[3])):
        assert abs(got - want) <= 0.05 * want


def _rr10_cases(lb, vn, g, dts=None):
    inflow = (1.0, 10.0, 0.0, 1.0 / 1.4)
    s2, s3, br = gasdyn.regular_reflection_states(1.4, inflow, 30.0)
    cases = [vn.case(g, (s[0], s[1], s[2], s[3] / s[0])) for s in (s2, s3)]
    return s2, s3, br, cases


def test_regular_reflection_mach10_at_paper_resolution():
    """Sec. 4.2 / Fig. 11 at the paper's size: 900 x 300, Mach-10 inflow, 30-degree
    incident shock, c1,c2,eta0 = 10,20,15, to t = 2.5 (FP32 storage). The time step is
    chosen by the GPU von Neumann scan (largest alpha = c2 dt/dx among the candidates
    that is strictly stable at both post-shock states over all modes of the grid); the
    run must reach a steady state whose plateaus behind the incident and the reflected
    shock match two-shock theory within 3% in density and pressure."""
    import paper_0706_0405_amd as lb
    from paper_0706_0405_amd import vn
    g0 = lb.Grid.from_workload(P.regular_reflection_paper())
    s2, s3, br, cases = _rr10_cases(lb, vn, g0)
    alphas = [0.025, 0.05, 0.075, 0.1, 0.15, 0.2, 0.25, 0.3]
    kx, ky = vn.modes(g0.nx, g0.ny)
    dts = vn.max_stable_dt(cases, [a * g0.dx / g0.c2 for a in alphas], kx, ky, 1e-12)
    alpha = round(min(dts) * g0.c2 / g0.dx, 6)
    say("scan-chosen alpha", alpha)
    assert alpha >= 0.05
    cfg = P.regular_reflection_paper(alpha=alpha)
    n = cfg["steps"]
    g, f = gpu_run(cfg, n, "f32")
    (rho, ux, uy, T), flags = gpu_fields(g, f, "f32")
    assert int(flags[0]) == 0, flags.tolist()
    fb = lb.empty(g, "f32", f.device)
    out = lb.run(g, f.clone(), fb, 100, n0=n, prec="f32")
    (rho2, _, _, _), _ = gpu_fields(g, out, "f32")
    resid = float((rho2 - rho).abs().sum() / rho.abs().sum())
    say("steady residual over 100 steps", resid)
    assert resid < 1e-8
    rho, T = rho.cpu().numpy(), T.cpu().numpy()
    p = rho * T
    theta = -math.degrees(math.atan2(s2[2], s2[1]))
    xw = g.ny * g.dx / math.tan(math.radians(30.0))
    assert (7.5 - xw) * math.tan(math.radians(br - theta)) > 0.45   # (7.5, 0.3) lies below the reflected shock
    r2, p2 = _patch(rho, 3.0, 2.5, g.dx), _patch(p, 3.0, 2.5, g.dx)
    r3, p3 = _patch(rho, 7.5, 0.3, g.dx), _patch(p, 7.5, 0.3, g.dx)
    say("region 2 rho %.4f (%.4f) p %.4f (%.4f); region 3 rho %.4f (%.4f) p %.4f (%.4f)"
        % (r2, s2[0], p2, s2[3], r3, s3[0], p3, s3[3]))
    for got, want in ((r2, s2[0]), (p2, s2[3]), (r3, s3[0]), (p3, s3[3])):
        assert abs(got - want) <= 0.03 * want


def test_regular_reflection_mach10_printed_time_step_is_unstable():
    """The printed dt = 1.5e-4 (alpha = 0.3): the scan finds the post-incident state
    unstable (radius > 1 + 1e-3) and the run goes non-finite before t = 2.5."""
    import paper_0706_0405_amd as lb
    from paper_0706_0405_amd import vn
    cfg = P.regular_reflection_paper(alpha=0.3)
    g = lb.Grid.from_workload(cfg)
    s2, s3, br, cases = _rr10_cases(lb, vn, g)
    kx, ky = vn.modes(g.nx, g.ny)
    r = vn.scan(cases, kx, ky, reduce=True).cpu()
    say("radius at alpha 0.3", r.tolist())
    assert float(r[0]) > 1 + 1e-3
    g, f = gpu_run(cfg, cfg["steps"], "f32")
    _, flags = gpu_fields(g, f, "f32")
    assert int(flags[0]) & 1, flags.tolist()


def test_double_mach_reflection_to_t_0_15():
    """Sec. 4.2 / Fig. 12 geometry (960 x 240, Mach-10 shock at 60 degrees to the wall,
    c1,c2,eta0 = 8,16,10) run to t = 0.15 in FP32 storage at alpha = 0.0125: positive
    density and temperature everywhere, the incident shock where the exact moving shock
    is (within 2 cells at three heights), and the undisturbed pre- and post-shock
    plateaus exact to 1e-3."""
    import paper_0706_0405_amd as lb
    cfg = P.double_mach(alpha=0.0125)
    g0 = lb.Grid.from_workload(cfg)
    n = int(round(0.15 / g0.dt))
    say("case double Mach to t = 0.15", n, "steps")
    g, f = gpu_run(cfg, n, "f32")
    (rho, ux, uy, T), flags = gpu_fields(g, f, "f32")
    assert int(flags[0]) == 0, flags.tolist()
    rho, T = rho.cpu().numpy(), T.cpu().numpy()
    p = rho * T
    post, t = cfg["post"], n * g.dt
    for y in (1.5, 2.0, 2.3):
        row = rho[int(round(y / g.dx - 0.5))]
        xs = (np.where(row > 0.5 * (cfg["pre"][0] + post[0]))[0].max() + 1) * g.dx
        xe = cfg["x0"] + y / math.tan(math.radians(60.0)) + 10.0 * t / math.sin(math.radians(60.0))
        say("shock at y = %.1f: %.3f (exact %.3f)" % (y, xs, xe))
        assert abs(xs - xe) <= 2 * g.dx
    for got, want in ((_patch(rho, 1.0, 2.0, g.dx), post[0]), (_patch(p, 1.0, 2.0, g.dx), post[3]),
                      (_patch(rho, 8.0, 1.0, g.dx), cfg["pre"][0]), (_patch(p, 8.0, 1.0, g.dx), cfg["pre"][3])):
        assert abs(got - want) <= 1e-3 * want


def test_double_mach_reflection_to_t_0_2_with_c1_above_the_wall_jet():
    """With the printed c1 = 8 the wall jet behind the Mach stem (|u| up to ~13 and more
    in its oscillations) outruns c1 and T turns negative at t ~ 0.19 (alpha = 0.0125);
    Sec. 3 (Fig. 7) finds u > c1 unstable and advises c1 about the largest flow speed.
    With c1,c2,eta0 = 16,32,20 the same problem runs to t = 0.2 at alpha = 0.05 with
    positive rho and T and the incident shock within 3 cells of the exact position."""
    import paper_0706_0405_amd as lb
    cfg = P.double_mach(alpha=0.05, c=(16.0, 32.0, 20.0))
    g0 = lb.Grid.from_workload(cfg)
    n = int(round(0.2 / g0.dt))
    say("case double Mach c1 = 16 to t = 0.2", n, "steps")
    g, f = gpu_run(cfg, n, "f32")
    (rho, ux, uy, T), flags = gpu_fields(g, f, "f32")
    assert int(flags[0]) == 0, flags.tolist()
    rho = rho.cpu().numpy()
    post, t = cfg["post"], n * g.dt
    say("wall jet max |u|", float(ux[0].abs().max()))
    for y in (1.5, 2.0, 2.3):
        row = rho[int(round(y / g.dx - 0.5))]
        xs = (np.where(row > 0.5 * (cfg["pre"][0] + post[0]))[0].max() + 1) * g.dx
        xe = cfg["x0"] + y / math.tan(math.radians(60.0)) + 10.0 * t / math.sin(math.radians(60.0))
        say("shock at y = %.1f: %.3f (exact %.3f)" % (y, xs, xe))
        assert abs(xs - xe) <= 3 * g.dx   # lambda = c1 dx is twice the printed one: a wider shock
