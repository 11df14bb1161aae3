"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: closed-form
moment identities, the printed (garbled) formulas failing where the readings
hold, invariants of the discrete map (uniform flow, conservation, mirror
symmetry, scale invariance), textbook reductions of the stencil, the
amplification matrix of Sec. 3 against the linearisation of the step itself,
the paper's qualitative stability claims, and exact Riemann solutions.
"""
import math
import os

import mpmath
import numpy as np

import pytest
import torch

from oracle import kt, scheme, vonneumann as vn
from workloads import gasdyn, problems as P

F64 = torch.float64
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_states(n, seed, umax=3.0):
    g = torch.Generator().manual_seed(seed)
    rho = 0.1 + 5 * torch.rand(n, generator=g, dtype=F64)
    ux = umax * (2 * torch.rand(n, generator=g, dtype=F64) - 1)
    uy = umax * (2 * torch.rand(n, generator=g, dtype=F64) - 1)
    T = 0.05 + 3 * torch.rand(n, generator=g, dtype=F64)
    return rho, ux, uy, T


PARAM_SETS = [(3.0, 9.0, 5.0, 1.4), (10.0, 20.0, 10.0, 1.4), (1.0, 3.0, 2.0, 5.0 / 3.0), (8.0, 16.0, 10.0, 1.4)]


# ------------------------------------------------------------------ velocity set / equilibrium

def test_velocity_set_geometry():
    """Eq. (e14) with the (cos, sin) reading: 4 axis speeds c1, 4 diagonal speeds c2, all distinct."""
    c1, c2 = 3.0, 9.0
    v = kt.velocities(c1, c2)
    assert v[0].abs().max() == 0
    s = c2 / math.sqrt(2.0)
    expect = [(0, 0), (-c1, 0), (0, -c1), (c1, 0), (0, c1), (-s, -s), (s, -s), (s, s), (-s, s)]
    assert torch.allclose(v, torch.tensor(expect, dtype=F64), rtol=0, atol=1e-14)
    # the printed (cos, cos) form would make velocities 5..8 collinear with (1,1)
    d = torch.cdist(v, v) + torch.eye(9, dtype=F64)
    assert d.min() > 0.5
    # exact symmetry of the set: every diagonal component is +-RN(c2/sqrt(2))
    mags = v[5:].abs().flatten().unique()
    assert mags.numel() == 1 and float(mags[0]) == float(mpmath.mpf(c2) / mpmath.sqrt(2))
    assert v[1:5].abs().sum(1).eq(c1).all()


@pytest.mark.parametrize("c1,c2,eta0,gamma", PARAM_SETS)
def test_equilibrium_moment_constraints(c1, c2, eta0, gamma):
    """The 10 scalar constraints Eqs. (e4)-(e8) on f_eq hold to round-off at random states."""
    rho, ux, uy, T = _rand_states(1000, 1)
    b = 2.0 / (gamma - 1.0)
    f = kt.feq(rho, ux, uy, T, c1, c2, eta0, gamma)
    s = c2 / math.sqrt(2.0)
    vx = torch.tensor([0, -c1, 0, c1, 0, -s, s, s, -s], dtype=F64)[:, None]
    vy = torch.tensor([0, 0, -c1, 0, c1, -s, -s, s, s], dtype=F64)[:, None]
    eta2 = torch.tensor([eta0 ** 2] + [0.0] * 8, dtype=F64)[:, None]
    usq = ux ** 2 + uy ** 2
    P_ = rho * T
    scale = rho * (b * T + usq + c2 ** 2)
    checks = [
        ((f).sum(0), rho),
        ((f * vx).sum(0), rho * ux),
        ((f * vy).sum(0), rho * uy),
        ((f * (vx ** 2 + vy ** 2 + eta2)).sum(0), rho * (b * T + usq)),
        ((f * vx * vx).sum(0), P_ + rho * ux * ux),
        ((f * vx * vy).sum(0), rho * ux * uy),
        ((f * vy * vx).sum(0), rho * uy * ux),
        ((f * vy * vy).sum(0), P_ + rho * uy * uy),
        ((f * (vx ** 2 + vy ** 2 + eta2) * vx).sum(0), rho * ((b + 2) * T + usq) * ux),
        ((f * (vx ** 2 + vy ** 2 + eta2) * vy).sum(0), rho * ((b + 2) * T + usq) * uy),
    ]
    for k, (got, want) in enumerate(checks):
        mult = (1.0 + usq.sqrt() + c2) if k >= 8 else 1.0
        err = ((got - want).abs() / (scale * mult)).max()
        assert err < 1e-13, (k, float(err))


def test_printed_forms_fail_the_constraints():
    """With the literal A_0 = (b-2)T/eta0 or the literal (cos, cos) velocities, mass/energy fail."""
    c1, c2, eta0, gamma = 3.0, 9.0, 5.0, 1.4
    b = 2.0 / (gamma - 1.0)
    rho, ux, uy, T = _rand_states(50, 2)
    usq = ux ** 2 + uy ** 2
    A, B, D = kt.coefficients(T, usq, c1, c2, eta0, b)
    v = kt.velocities(c1, c2)
    # literal A_0
    A_lit = [(b - 2.0) * T / eta0] + A[1:]
    mass = sum(rho * (A_lit[i] + B[i] * (v[i, 0] * ux + v[i, 1] * uy) + D[i] * (v[i, 0] * ux + v[i, 1] * uy) ** 2)
               for i in range(9))
    assert ((mass - rho).abs() / rho).max() > 1e-2
    # literal (cos, cos) for the diagonal group
    vl = v.clone()
    for i in range(5, 9):
        th = math.pi * ((i + 1) / 2.0 + 0.25)
        vl[i, 0] = vl[i, 1] = c2 * math.cos(th)
    mom = sum(rho * (A[i] + B[i] * (vl[i, 0] * ux + vl[i, 1] * uy) + D[i] * (vl[i, 0] * ux + vl[i, 1] * uy) ** 2)
              * vl[i, 0] for i in range(9))
    assert ((mom - rho * ux).abs() / rho).max() > 1e-2


@pytest.mark.parametrize("c1,c2,eta0,gamma", PARAM_SETS)
def test_moments_invert_equilibrium(c1, c2, eta0, gamma):
    rho, ux, uy, T = _rand_states(1000, 3)
    f = kt.feq(rho, ux, uy, T, c1, c2, eta0, gamma)
    r, u, v, t = kt.moments(f, c1, c2, eta0, gamma)
    assert ((r - rho).abs() / rho).max() < 1e-13
    assert (u - ux).abs().max() < 1e-13 * (1 + c2)
    assert (v - uy).abs().max() < 1e-13 * (1 + c2)
    assert ((t - T).abs() / (T + ux ** 2 + uy ** 2)).max() < 1e-13


def test_collision_jacobian_is_rank4_projection():
    """J = d f_eq / d f is idempotent with eigenvalues {1 x4, 0 x5} (f_eq depends on f only via 4 moments)."""
    J = vn.collision_jacobian(1.0, 10.0, 0.0, 1.0, 10.0, 20.0, 10.0, 1.4)
    assert (J @ J - J).abs().max() < 1e-12 * J.abs().max()
    ev = torch.linalg.eigvals(J)
    ones = (ev - 1).abs() < 1e-10
    zeros = ev.abs() < 1e-10
    assert int(ones.sum()) == 4 and int(zeros.sum()) == 5


def test_mirror_permutations():
    """A y-normal wall swaps 2<->4, 5<->8, 6<->7; an x-normal wall swaps 1<->3, 5<->6, 7<->8."""
    assert kt.mirror_permutation(3, 9, 1) == [0, 1, 4, 3, 2, 8, 7, 6, 5]
    assert kt.mirror_permutation(3, 9, 0) == [0, 3, 2, 1, 4, 6, 5, 8, 7]


# ------------------------------------------------------------------ step invariants

def _uniform(pb, state):
    r, u, v, p = state
    shape = (pb.ny, pb.nx)
    return scheme.init(pb, torch.full(shape, r, dtype=F64), torch.full(shape, u, dtype=F64),
                       torch.full(shape, v, dtype=F64), torch.full(shape, p, dtype=F64))


@pytest.mark.parametrize("kind", ["periodic", "inflow"])
def test_uniform_flow_is_stationary(kind):
    st = (1.3, 0.7, -0.4, 0.9)
    cfg = P.periodic_smooth(nx=12, ny=8)
    if kind == "inflow":
        cfg["edges"] = [{"kind": "inflow", "a": st} for _ in range(4)]
    pb = scheme.Problem.from_dict(cfg)
    f0 = _uniform(pb, st)
    f1 = scheme.run(pb, f0, 5)
    assert ((f1 - f0).abs() / f0.abs().max()).max() < 1e-15 * 8


def test_conservation_on_periodic_grid():
    """Mass, momentum and energy totals are invariant on a periodic grid (zero-sum stencils,
    moment-preserving collisions), to 1e-12 relative over 1000 steps."""
    cfg = P.periodic_smooth(nx=16, ny=12)
    pb = scheme.Problem.from_dict(cfg)
    f = scheme.init(pb, *P.init_fields(cfg))
    tot0 = [float(q.sum()) for q in kt.conserved(f, pb.c1, pb.c2, pb.eta0)]
    f = scheme.run(pb, f, 1000)
    tot1 = [float(q.sum()) for q in kt.conserved(f, pb.c1, pb.c2, pb.eta0)]
    scale = [abs(tot0[0]), abs(tot0[0]) * pb.c1, abs(tot0[0]) * pb.c1, abs(tot0[3])]
    for a, b, s in zip(tot0, tot1, scale):
        assert abs(a - b) / s < 1e-12, (a, b)
    assert torch.isfinite(f).all()


def test_scale_invariance():
    """(dx, dt) -> (s dx, s dt) with lambda per Eq. (SEC-VON-13) leaves the grid map unchanged."""
    cfg = P.periodic_smooth(nx=12, ny=10)
    fields = P.init_fields(cfg)
    pb1 = scheme.Problem.from_dict(cfg)
    cfg2 = dict(cfg, dx=cfg["dx"] * 4.0, dt=cfg["dt"] * 4.0)
    pb2 = scheme.Problem.from_dict(cfg2)
    f1 = scheme.run(pb1, scheme.init(pb1, *fields), 20)
    f2 = scheme.run(pb2, scheme.init(pb2, *fields), 20)
    assert ((f1 - f2).abs().max() / f1.abs().max()) < 1e-14


def test_wall_equals_mirror_symmetric_periodic_domain():
    """A channel between two reflecting walls equals half of a periodic domain holding the
    mirror image of the data (walls on cell faces)."""
    cfg = P.periodic_smooth(nx=10, ny=6)
    pb_half = scheme.Problem.from_dict(dict(cfg, edges=[{"kind": "periodic"}, {"kind": "periodic"},
                                                        {"kind": "wall"}, {"kind": "wall"}]))
    pb_full = scheme.Problem.from_dict(dict(cfg, ny=12))
    f_half = scheme.init(pb_half, *P.init_fields(cfg))
    perm = kt.mirror_permutation(pb_half.c1, pb_half.c2, 1)
    mirrored = f_half[perm].flip(1)
    f_full = torch.cat([f_half, mirrored], 1)
    h = scheme.run(pb_half, f_half, 30)
    full = scheme.run(pb_full, f_full, 30)
    assert ((h - full[:, :6]).abs().max() / h.abs().max()) < 1e-14


def _step_jacobian(pb, f0, n=0):
    flat = f0.reshape(-1)

    def g(x):
        return scheme.step(pb, x.reshape(f0.shape), n).reshape(-1)

    return torch.autograd.functional.jacobian(g, flat, vectorize=True)


@pytest.mark.parametrize("beta,expect", [(0.0, "upwind"), (0.5, "central"), (0.25, "mixed")])
def test_stencil_reductions(beta, expect):
    """Neighbour coefficients of the linearised step: beta = 0 is first-order upwind,
    beta = 0.5 is central differencing (Sec. 2, after Eqs. (SEC-VON-2a/2b)), plus lambda dt/dx^2."""
    cfg = P.periodic_smooth(nx=5, ny=5)
    cfg["beta"] = beta
    pb = scheme.Problem.from_dict(cfg)
    f0 = _uniform(pb, (1.0, 0.3, 0.1, 1.0))
    J = _step_jacobian(pb, f0).reshape(9, 5, 5, 9, 5, 5)
    v = kt.velocities(pb.c1, pb.c2)
    r = pb.dt / pb.dx
    for i in range(9):
        vx = float(v[i, 0])
        lam = pb.lam[i] * pb.dt / pb.dx ** 2
        down = J[i, 2, 2, i, 2, 3]   # d f_i'(x) / d f_i(x + dx)
        up = J[i, 2, 2, i, 2, 1]     # d f_i'(x) / d f_i(x - dx)
        if vx == 0:
            assert abs(float(down) - lam) < 1e-14 and abs(float(up) - lam) < 1e-14
            continue
        a = abs(vx) * r
        if expect == "upwind":
            want_up, want_down = (a, 0.0) if vx > 0 else (0.0, a)
        elif expect == "central":
            want_up, want_down = (a / 2, -a / 2) if vx > 0 else (-a / 2, a / 2)
        else:
            want_up, want_down = ((1 - beta) * a, -beta * a) if vx > 0 else (-beta * a, (1 - beta) * a)
        assert abs(float(up) - (want_up + lam)) < 1e-13, (i, float(up), want_up + lam)
        assert abs(float(down) - (want_down + lam)) < 1e-13, (i, float(down), want_down + lam)


@pytest.mark.parametrize("tau", [1.0, 2.0])
def test_amplification_matrix_matches_step_linearisation(tau):
    """The spectrum of the one-step Jacobian on an N x N periodic grid equals the union of
    eig G(2 pi (p, q)/N), Eqs. (SEC-VON-8), (SEC-VON-9), (SEC-VON-12)."""
    N = 6
    cfg = P.periodic_smooth(nx=N, ny=N, c=(10.0, 20.0, 10.0), alpha=0.3)
    cfg["tau"] = tau
    pb = scheme.Problem.from_dict(cfg)
    state = (1.0, 4.0, -1.5, 1.2)
    f0 = _uniform(pb, state)
    J = _step_jacobian(pb, f0)
    ev_step = torch.linalg.eigvals(J)
    params = {"c1": pb.c1, "c2": pb.c2, "eta0": pb.eta0, "gamma": pb.gamma, "tau": tau,
              "beta": pb.beta, "dt": pb.dt, "dx": pb.dx, "lam": pb.lam}
    r, u, v, p = state
    Jc = vn.collision_jacobian(r, u, v, p / r, pb.c1, pb.c2, pb.eta0, pb.gamma)
    ev_g = []
    for p_ in range(N):
        for q in range(N):
            G = vn.amplification((r, u, v, p / r), params, 2 * math.pi * p_ / N, 2 * math.pi * q / N, Jc)
            ev_g.append(torch.linalg.eigvals(G))
    ev_g = torch.cat(ev_g)
    assert ev_g.numel() == ev_step.numel()
    d1 = (ev_step[:, None] - ev_g[None, :]).abs().min(1).values.max()
    d2 = (ev_g[:, None] - ev_step[None, :]).abs().min(1).values.max()
    assert d1 < 1e-10 and d2 < 1e-10


def _claims():
    rows = []
    for line in open(os.path.join(GOLDEN, "vonneumann_claims.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


@pytest.mark.parametrize("row", _claims(), ids=lambda r: "-".join(r))
def test_vonneumann_figure_claims(row):
    fig = row[0]
    state = [1.0, 10.0, 0.0, 1.0]  # rho, u1, u2, T
    kw = {}
    if fig == "fig2":
        kw["dissipation"] = (row[2] == "on")
        alpha, expect = float(row[3]), row[4]
    else:
        name, val, alpha, expect = row[1], float(row[2]), float(row[3]), row[4]
        if name == "eta0":
            kw["eta0"] = val
        elif name == "T":
            state[3] = val
        elif name == "u1":
            state[1] = val
    params = vn.figure_params(alpha=alpha, **kw)
    ks, m = vn.scan_diagonal(tuple(state), params)
    mx = max(m)
    if expect == "stable":
        assert mx <= 1 + 1e-9, mx
    elif expect == "unstable":
        assert mx > 1 + 1e-3, mx
    else:
        kmax = ks[max(range(len(m)), key=lambda j: m[j])]
        assert 1 + 1e-4 < mx < 1.05 and abs(kmax - 0.5) < 0.15, (mx, kmax)


# ------------------------------------------------------------------ exact solutions

def _riemann_l1(cfg):
    pb = scheme.Problem.from_dict(cfg)
    f = scheme.run(pb, scheme.init(pb, *P.init_fields(cfg)), cfg["steps"])
    rho = scheme.fields(pb, f)[0][0]
    L, R = cfg["left"], cfg["right"]
    xc = [(i + 0.5) * pb.dx for i in range(pb.nx)]
    er, _, _ = gasdyn.riemann_cell_average(pb.gamma, (L[0], L[1], L[3]), (R[0], R[1], R[3]),
                                           cfg["x_disc"], cfg["steps"] * pb.dt, xc, pb.dx)
    er = torch.tensor(er, dtype=F64)
    return float((rho - er).abs().sum() / er.abs().sum()), f


def test_sod_against_exact_solution_and_refinement():
    errs = []
    for nx, steps in ((200, 500), (400, 1000), (800, 2000)):
        cfg = P.sod(nx=nx, ny=1, steps=steps)
        e, f = _riemann_l1(cfg)
        assert torch.isfinite(f).all()
        errs.append(e)
    assert errs[0] < 0.06, errs
    assert errs[0] > errs[1] > errs[2], errs


@pytest.mark.slow
def test_ratio1000_against_exact_solution():
    cfg = P.ratio1000(ny=1)
    e, f = _riemann_l1(cfg)
    assert e < 0.02, e


def test_exact_riemann_solver_jump_conditions():
    """The star states satisfy the Rankine-Hugoniot conditions across each shock and
    isentropy + the Riemann invariant across each rarefaction."""
    g = 1.4
    for left, right in (((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)), ((1000.0, 0.0, 1000.0), (1.0, 0.0, 1.0)),
                        ((1.4, 30.0, 1.0), (1.4, 0.0, 1.0)), ((1.0, -2.0, 0.4), (1.0, 2.0, 0.4))):
        st = gasdyn.riemann_star(g, left, right)
        for side, (r0, u0, p0), rs in (("L", left, st.rho_l), ("R", right, st.rho_r)):
            shock = st.left_shock if side == "L" else st.right_shock
            c0 = math.sqrt(g * p0 / r0)
            if shock:
                # shock speed from mass conservation, then momentum and energy fluxes must match
                S = (rs * st.u - r0 * u0) / (rs - r0)
                E0 = p0 / (g - 1) + 0.5 * r0 * u0 ** 2
                Es = st.p / (g - 1) + 0.5 * rs * st.u ** 2
                mom = (rs * st.u ** 2 + st.p) - (r0 * u0 ** 2 + p0) - S * (rs * st.u - r0 * u0)
                en = (st.u * (Es + st.p)) - (u0 * (E0 + p0)) - S * (Es - E0)
                assert abs(mom) < 1e-9 * (r0 * u0 ** 2 + p0 + st.p + 1)
                assert abs(en) < 1e-9 * (abs(u0 * (E0 + p0)) + abs(st.u * (Es + st.p)) + 1)
            else:
                assert abs(st.p / rs ** g - p0 / r0 ** g) < 1e-10 * p0 / r0 ** g
                cs = math.sqrt(g * st.p / rs)
                sgn = 1.0 if side == "L" else -1.0
                assert abs((st.u + sgn * 2 * cs / (g - 1)) - (u0 + sgn * 2 * c0 / (g - 1))) < 1e-10 * (1 + c0)


def test_exact_riemann_sod_textbook_values():
    """Sod problem star region: p* = 0.30313, u* = 0.92745 (Toro, Riemann Solvers and
    Numerical Methods for Fluid Dynamics, Sec. 4.3, test 1)."""
    st = gasdyn.riemann_star(1.4, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    assert abs(st.p - 0.30313) < 5e-6 and abs(st.u - 0.92745) < 5e-6


def test_oblique_shock_reproduces_paper_top_state():
    """Eq. (Riemann-3): the printed top state is the oblique-shock state of the Mach-10 inflow."""
    rows = {}
    for line in open(os.path.join(GOLDEN, "regular_reflection_top_state.txt")):
        if line.strip() and not line.startswith("#"):
            k, *vals = line.split()
            rows[k] = [float(x) for x in vals]
    got = gasdyn.oblique_shock_state(1.4, tuple(rows["inflow"]), 30.0)
    for a, b in zip(got, rows["top"]):
        assert abs(a - b) <= 0.6e-4 * max(1.0, abs(b)), (got, rows["top"])


def test_normal_shock_mach10():
    """Mach-10 normal shock into (1.4, 0, 0, 1): rho = 8, p = 116.5, |u| = 8.25."""
    r, u, v, p = gasdyn.moving_shock_post_state(1.4, (1.4, 1.0), 10.0, -30.0)
    assert abs(r - 8.0) < 1e-12 and abs(p - 116.5) < 1e-10
    assert abs(math.hypot(u, v) - 8.25) < 1e-12 and abs(math.degrees(math.atan2(v, u)) + 30.0) < 1e-10


def test_regular_reflection_two_shock_theory():
    """Behind the reflected shock the flow is parallel to the wall and the shock is attached."""
    s2, s3, br = gasdyn.regular_reflection_states(1.4, (1.0, 2.9, 0.0, 1.0 / 1.4), 30.0)
    assert s3[2] == 0.0 and s3[1] > 0 and s3[0] > s2[0] > 1.0 and s3[3] > s2[3]
    th = -math.degrees(math.atan2(s2[2], s2[1]))
    m2 = math.hypot(s2[1], s2[2]) / math.sqrt(1.4 * s2[3] / s2[0])
    assert abs(gasdyn.deflection_angle_deg(1.4, m2, br) - th) < 1e-9


def test_shock_edge_behind_and_ahead():
    """The moving-shock edge gives f_eq(a) behind and f_eq(b) ahead of x0 + y/tan + s t/sin."""
    cfg = P.double_mach(nx=48, ny=12)
    pb = scheme.Problem.from_dict(cfg)
    f = scheme.init(pb, *P.init_fields(cfg))
    t = 37 * pb.dt
    F = scheme.pad(pb, f, t)
    fa = scheme.feq_state(pb, cfg["post"])
    fb = scheme.feq_state(pb, cfg["pre"])
    yg = (pb.ny + 0.5) * pb.dx
    xs = cfg["x0"] + yg / math.tan(math.radians(60)) + 10.0 * t / math.sin(math.radians(60))
    for i in range(pb.nx):
        want = fa if (i + 0.5) * pb.dx < xs else fb
        assert torch.equal(F[:, pb.ny + 1, i + 1], want)
    # bottom: inflow ahead of the wall start, mirror image beyond it
    perm = kt.mirror_permutation(pb.c1, pb.c2, 1)
    for i in range(pb.nx):
        want = fa if i < pb.edges[2].split else f[perm, 0, i]
        assert torch.equal(F[:, 0, i + 1], want)


# ------------------------------------------------------------------ moving-shock edge against the interior shock

def _free_shock_problem(nx=72, ny=24):
    """The double-Mach shock (Mach 10 at 60 degrees into (1.4, 0, 0, 1), Sec. 4.2) with no
    wall: both y edges are the moving-shock edge, so the exact solution is the initial
    planar shock translated along its normal."""
    cfg = P.double_mach(nx=nx, ny=ny, length=nx * 0.01, wall_cells=10, alpha=0.1)
    top = cfg["edges"][3]
    cfg["edges"] = [cfg["edges"][0], cfg["edges"][1], dict(top), dict(top)]
    return cfg


def _equal_area_positions(rho, pre, post, k0, dx):
    """Per row, the x where a sharp jump from post to pre would hold the same mass as
    the row right of face k0 (behind the shock the row is at the post-shock state)."""
    return (k0 + (rho[:, k0:] - pre).sum(1) / (post - pre)) * dx


def _ghost_transition(pb, f, name, t, pre, post):
    """x of the cell face where the ghost row of edge `name` switches from the
    post-shock to the pre-shock equilibrium (its density, Eq. (e4))."""
    r = scheme._ghost_line(pb, f, name, t).sum(0)
    k = torch.nonzero(r > 0.5 * (pre + post)).max()
    return (int(k) + 1) * pb.dx


def _shock_pin(cfg, plant=None):
    """Run the oracle until the shock has moved 25 cells; return the measured
    deviations of the interior shock from planar-shock physics and of the ghost
    transitions from the interior shock line. plant = (field, fn) changes that
    parameter of the two shock ghost edges only (a planted mistake)."""
    pre, post = cfg["pre"], cfg["post"]
    pb = scheme.Problem.from_dict(cfg)
    if plant:
        for e in pb.edges[2:]:
            setattr(e, plant[0], plant[1](getattr(e, plant[0])))
    fields = P.init_fields(cfg)
    nx, ny, dx = pb.nx, pb.ny, pb.dx
    slope = 1.0 / math.tan(math.radians(60.0))           # x per unit y along the incident shock
    # Rankine-Hugoniot: the shock speed along its normal n (towards the gas at rest) is the
    # jump of the mass flux over the jump of the density
    n = torch.tensor([1.0, -slope], dtype=torch.float64) / math.sqrt(1.0 + slope * slope)
    un_post = post[1] * float(n[0]) + post[2] * float(n[1])
    un_pre = pre[1] * float(n[0]) + pre[2] * float(n[1])
    speed = (post[0] * un_post - pre[0] * un_pre) / (post[0] - pre[0])
    shift = 25.0 * dx                                      # x displacement to run for
    nsteps = int(round(shift / (speed * pb.dt * math.sqrt(1.0 + slope * slope))))
    y = (torch.arange(ny, dtype=torch.float64) + 0.5) * dx
    x_init = _equal_area_positions(torch.as_tensor(fields[0]), pre[0], post[0], 4, dx)
    f = scheme.init(pb, *fields)
    for k in range(nsteps):
        f = scheme.step(pb, f, k)
    t = nsteps * pb.dt
    x_end = _equal_area_positions(scheme.fields(pb, f)[0], pre[0], post[0], 4, dx)
    inner = slice(2, ny - 2)                               # rows clear of the ghost rows' own stencil
    A = torch.stack([torch.ones(ny, dtype=torch.float64), y], 1)[inner]
    a0 = float(torch.linalg.lstsq(A, x_init[inner].unsqueeze(1)).solution[0])
    a1, b1 = [float(v) for v in torch.linalg.lstsq(A, x_end[inner].unsqueeze(1)).solution[:, 0]]
    resid = float((x_end[inner] - (a1 + b1 * y[inner])).abs().max()) / dx
    moved = (a1 - a0) / dx
    want = speed * t * math.sqrt(1.0 + slope * slope) / dx
    gb = _ghost_transition(pb, f, "y-", t, pre[0], post[0])
    gt = _ghost_transition(pb, f, "y+", t, pre[0], post[0])
    dev_b = (gb - (a1 + b1 * (-0.5 * dx))) / dx
    dev_t = (gt - (a1 + b1 * ((ny + 0.5) * dx))) / dx
    return {"speed": speed, "moved": moved, "want": want, "slope_err": abs(b1 - slope), "resid": resid,
            "ghost_dev": max(abs(dev_b), abs(dev_t))}


def _shock_pin_holds(d):
    """Planar-shock physics in the interior and ghosts on the interior shock line:
    straight (0.3 cell), at the initial 60 degrees (slope within 0.012), moved by the
    Rankine-Hugoniot speed times t (0.3 cell), ghost transitions within 0.6 cell of
    the line extended to the ghost rows."""
    return d["resid"] <= 0.3 and d["slope_err"] <= 0.012 and abs(d["moved"] - d["want"]) <= 0.3 \
        and d["ghost_dev"] <= 0.6


def test_moving_shock_edge_moves_with_the_interior_shock():
    """The moving-shock ghost rows, checked against the dynamics instead of their
    formula: on a domain whose y edges are both moving-shock edges, the interior shock
    (equal-area position per row, which a conservative scheme moves at the
    Rankine-Hugoniot speed) must stay planar at 60 degrees, move by the speed the
    mass-flux jump of the two states gives, and pass through the ghost rows' transitions."""
    nthreads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        d = _shock_pin(_free_shock_problem())
    finally:
        torch.set_num_threads(nthreads)
    assert abs(d["speed"] - 10.0) < 1e-9          # the states are a Mach-10 shock
    assert d["want"] > 24.0
    assert _shock_pin_holds(d), d


@pytest.mark.parametrize("plant", [("speed", 0.9), ("speed", 1.05), ("angle_deg", -3.0), ("angle_deg", 1.0),
                                   ("x0", 0.02), ("x0", -0.01)], ids=lambda p: "%s%+g" % p)
def test_moving_shock_pin_catches_planted_ghost_mistakes(plant):
    """The pin above fails when the ghost rows alone are moved: a speed off by 5-10%,
    the angle off by 1-3 degrees, the origin off by one or two cells."""
    field, v = plant
    fn = (lambda s: s * v) if field == "speed" else (lambda s: s + v)
    nthreads = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        d = _shock_pin(_free_shock_problem(), (field, fn))
    finally:
        torch.set_num_threads(nthreads)
    assert not _shock_pin_holds(d), d


def test_amplification_over_many_wave_vectors_equals_the_single_form():
    """The vectorised G(k) equals the per-wave-vector G of Eqs. (SEC-VON-8), (SEC-VON-9),
    (SEC-VON-12) (pinned above against the step's linearisation) at random states,
    parameters and wave vectors, bitwise; its largest radius too."""
    rng = np.random.default_rng(11)
    for _ in range(5):
        c1 = float(rng.uniform(1, 10))
        p = vn.figure_params(c1=c1, c2=c1 * float(rng.uniform(1.5, 3)), eta0=c1 * float(rng.uniform(1, 2)),
                             alpha=float(rng.uniform(0.05, 0.4)), beta=float(rng.uniform(0, 0.5)),
                             tau=float(rng.uniform(0.8, 2)))
        st = (float(rng.uniform(0.5, 2)), float(rng.uniform(-c1, c1)), float(rng.uniform(-c1, c1) / 3),
              float(rng.uniform(0.2, 1) * c1 * c1 / 4))
        kx = rng.uniform(-math.pi, math.pi, 7).tolist()
        ky = rng.uniform(-math.pi, math.pi, 7).tolist()
        G = vn.amplification_many(st, p, kx, ky)
        for q in range(7):
            assert torch.equal(G[q], vn.amplification(st, p, kx[q], ky[q]))
        assert vn.max_modulus_many(st, p, kx, ky) == max(vn.max_modulus(st, p, a, b) for a, b in zip(kx, ky))


def test_fp32_storage_run_rounds_each_stored_state():
    """scheme.run with float32 storage equals FP64 steps with each result rounded to the
    nearest float32 (round-to-nearest is exact in float64 and idempotent), and differs
    from the FP64 run by about the float32 rounding."""
    cfg = P.periodic_smooth(nx=20, ny=8, steps=5)
    pb = scheme.Problem.from_dict(cfg)
    f0 = scheme.store(scheme.init(pb, *P.init_fields(cfg)), torch.float32)
    assert torch.equal(scheme.store(f0, torch.float32), f0)
    f = f0
    for n in range(5):
        f = scheme.step(pb, f, n).to(torch.float32).to(torch.float64)
    got = scheme.run(pb, f0, 5, storage=torch.float32)
    assert torch.equal(got, f)
    f64 = scheme.run(pb, f0, 5)
    rel = float(((got - f64).abs() / f64.abs()).max())
    assert 0 < rel < 5 * 2.0 ** -24
