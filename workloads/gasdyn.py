"""Ideal-gas relations used to *define* workloads (boundary states, batch draws).

These are textbook gas-dynamics closed forms, not part of the lattice Boltzmann
method: normal and oblique shock (Rankine-Hugoniot) relations and the exact
solution of the 1D Riemann problem for the Euler equations (the target
equations of the kinetic model, Sec. 2, Eq. (e2), with P = rho*T, R = 1).
They build the inflow states of the shock-reflection problems (Sec. 4.2,
Eq. (Riemann-3)) and the star states that bound the velocity range of a
batched Riemann draw, and they give the exact solutions the validation runs of
Sec. 4.1 are compared with.

Neither the GPU path nor the CPU oracle implements any of this arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


# ---------------------------------------------------------------- shocks

def normal_shock_ratios(gamma: float, mach: float):
    """Density, pressure ratio across a normal shock of upstream normal Mach `mach`.

    rho2/rho1 = (g+1) M^2 / ((g-1) M^2 + 2);  p2/p1 = 1 + 2g/(g+1) (M^2 - 1).
    """
    m2 = mach * mach
    rr = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    pr = 1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0)
    return rr, pr


def oblique_shock_state(gamma: float, upstream, wave_angle_deg: float):
    """State behind a straight oblique shock of wave angle `wave_angle_deg`.

    `upstream` = (rho, ux, 0, p) with the flow along +x. The shock is inclined
    so that it turns the flow towards -y (the incident shock of a regular
    reflection off a wall at the bottom, Sec. 4.2). Returns (rho, ux, uy, p).
    """
    rho1, u1, v1, p1 = upstream
    if v1 != 0.0:
        raise ValueError("upstream flow must be along +x")
    b = math.radians(wave_angle_deg)
    c1 = math.sqrt(gamma * p1 / rho1)
    mn = u1 * math.sin(b) / c1
    if mn <= 1.0:
        raise ValueError("normal Mach number must exceed 1")
    rr, pr = normal_shock_ratios(gamma, mn)
    un1 = u1 * math.sin(b)
    ut = u1 * math.cos(b)
    un2 = un1 / rr
    # tangent t = (cos b, -sin b), normal n = (sin b, cos b)
    ux = ut * math.cos(b) + un2 * math.sin(b)
    uy = -ut * math.sin(b) + un2 * math.cos(b)
    return (rho1 * rr, ux, uy, p1 * pr)


def deflection_angle_deg(gamma: float, mach: float, wave_angle_deg: float) -> float:
    """Flow deflection across an oblique shock (theta-beta-M relation)."""
    b = math.radians(wave_angle_deg)
    m2 = mach * mach
    num = 2.0 / math.tan(b) * (m2 * math.sin(b) ** 2 - 1.0)
    den = m2 * (gamma + math.cos(2.0 * b)) + 2.0
    return math.degrees(math.atan(num / den))


def wave_angle_for_deflection(gamma: float, mach: float, theta_deg: float) -> float:
    """Weak-branch wave angle (deg) that deflects a Mach `mach` flow by theta."""
    mu = math.degrees(math.asin(1.0 / mach))
    # bracket the weak solution between the Mach angle and the max-deflection angle
    lo, hi = mu + 1e-12, mu
    best, bmax = -1.0, mu
    for k in range(1, 9000):
        bb = mu + (90.0 - mu) * k / 9000.0
        d = deflection_angle_deg(gamma, mach, bb)
        if d > best:
            best, bmax = d, bb
    if theta_deg > best:
        raise ValueError("deflection exceeds the attached-shock maximum")
    lo, hi = mu + 1e-12, bmax
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if deflection_angle_deg(gamma, mach, mid) < theta_deg:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def regular_reflection_states(gamma: float, upstream, wave_angle_deg: float):
    """Two-shock theory of a regular reflection off a flat wall along +x.

    Returns (state2, state3, reflected_wave_angle_deg_relative_to_flow2):
    state2 behind the incident shock, state3 behind the reflected shock, whose
    flow is parallel to the wall again.
    """
    s2 = oblique_shock_state(gamma, upstream, wave_angle_deg)
    rho2, u2, v2, p2 = s2
    q2 = math.hypot(u2, v2)
    m2 = q2 / math.sqrt(gamma * p2 / rho2)
    theta = -math.degrees(math.atan2(v2, u2))  # deflection to undo
    br = wave_angle_for_deflection(gamma, m2, theta)
    mn = m2 * math.sin(math.radians(br))
    rr, pr = normal_shock_ratios(gamma, mn)
    # speed behind the reflected shock, flow along +x
    b = math.radians(br)
    un2 = q2 * math.sin(b) / rr
    ut = q2 * math.cos(b)
    q3 = math.hypot(un2, ut)
    return s2, (rho2 * rr, q3, 0.0, p2 * pr), br


def moving_shock_post_state(gamma: float, pre, mach: float, direction_deg: float):
    """State behind a normal shock of Mach `mach` running into gas at rest.

    `pre` = (rho, p) of the quiescent gas; the shock moves along the unit
    vector at `direction_deg` from +x. Returns (rho, ux, uy, p).
    """
    rho1, p1 = pre
    c1 = math.sqrt(gamma * p1 / rho1)
    rr, pr = normal_shock_ratios(gamma, mach)
    w = mach * c1 * (1.0 - 1.0 / rr)
    a = math.radians(direction_deg)
    return (rho1 * rr, w * math.cos(a), w * math.sin(a), p1 * pr)


# ---------------------------------------------------------------- exact Riemann solver

@dataclass
class RiemannStar:
    p: float
    u: float
    rho_l: float
    rho_r: float
    left_shock: bool
    right_shock: bool


def _pressure_fn(p, rho, pk, ck, gamma):
    """Textbook pressure function f_K(p) and its derivative (shock or rarefaction)."""
    if p > pk:
        a = 2.0 / ((gamma + 1.0) * rho)
        b = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (b + p))
    e = (gamma - 1.0) / (2.0 * gamma)
    r = p / pk
    return 2.0 * ck / (gamma - 1.0) * (r ** e - 1.0), 1.0 / (rho * ck) * r ** (-(gamma + 1.0) / (2.0 * gamma))


def riemann_star(gamma: float, left, right) -> RiemannStar:
    """Star-region pressure and velocity of the exact Riemann solution.

    `left`/`right` = (rho, u, p). Raises ValueError when the data create vacuum.
    """
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    if ur - ul >= 2.0 * (cl + cr) / (gamma - 1.0):
        raise ValueError("initial data generate vacuum")
    # two-rarefaction guess, then Newton, then bisection safeguard
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((cl + cr - 0.5 * (gamma - 1.0) * (ur - ul)) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-14 * max(pl, pr))
    for _ in range(100):
        fl, dl = _pressure_fn(p, rl, pl, cl, gamma)
        fr, dr = _pressure_fn(p, rr, pr, cr, gamma)
        g = fl + fr + ur - ul
        pn = p - g / (dl + dr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_fn(p, rl, pl, cl, gamma)
    fr, _ = _pressure_fn(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    if p > pl:
        rho_l = rl * (p / pl + g1) / (g1 * p / pl + 1.0)
    else:
        rho_l = rl * (p / pl) ** (1.0 / gamma)
    if p > pr:
        rho_r = rr * (p / pr + g1) / (g1 * p / pr + 1.0)
    else:
        rho_r = rr * (p / pr) ** (1.0 / gamma)
    return RiemannStar(p, u, rho_l, rho_r, p > pl, p > pr)


def riemann_sample(gamma: float, left, right, xi):
    """Exact solution (rho, u, p) at similarity coordinates xi = (x - x0)/t.

    `xi` is an iterable of floats; returns three lists.
    """
    rl, ul, pl = left
    rr, ur, pr = right
    st = riemann_star(gamma, left, right)
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    g = gamma
    out_r, out_u, out_p = [], [], []
    for s in xi:
        if s <= st.u:  # left of contact
            if st.left_shock:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * st.p / pl + (g - 1) / (2 * g))
                val = (rl, ul, pl) if s <= sl else (st.rho_l, st.u, st.p)
            else:
                shl = ul - cl
                cml = cl * (st.p / pl) ** ((g - 1) / (2 * g))
                stl = st.u - cml
                if s <= shl:
                    val = (rl, ul, pl)
                elif s >= stl:
                    val = (st.rho_l, st.u, st.p)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    rho = rl * (c / cl) ** (2 / (g - 1))
                    val = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if st.right_shock:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * st.p / pr + (g - 1) / (2 * g))
                val = (rr, ur, pr) if s >= sr else (st.rho_r, st.u, st.p)
            else:
                shr = ur + cr
                cmr = cr * (st.p / pr) ** ((g - 1) / (2 * g))
                str_ = st.u + cmr
                if s >= shr:
                    val = (rr, ur, pr)
                elif s <= str_:
                    val = (st.rho_r, st.u, st.p)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    rho = rr * (c / cr) ** (2 / (g - 1))
                    val = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
        out_r.append(val[0])
        out_u.append(val[1])
        out_p.append(val[2])
    return out_r, out_u, out_p


def riemann_cell_average(gamma, left, right, x0, t, xcenters, dx, sub=16):
    """Exact solution averaged over cells of width dx (midpoint sub-sampling)."""
    xi = []
    for xc in xcenters:
        for k in range(sub):
            x = xc - 0.5 * dx + (k + 0.5) * dx / sub
            xi.append((x - x0) / t)
    r, u, p = riemann_sample(gamma, left, right, xi)
    n = len(xcenters)
    avg = lambda a: [sum(a[i * sub:(i + 1) * sub]) / sub for i in range(n)]
    return avg(r), avg(u), avg(p)
