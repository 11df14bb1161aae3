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
