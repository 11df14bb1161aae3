"""Finite-difference LB time step with the added dissipation (oracle; test infrastructure only).

One step, Eq. (SEC-VON-11) solved for f(x, t + dt) with the relaxation time in
units of dt (the paper sets dt equal to the Knudsen number, Eq. (SEC-VON-1)):

  f_i' = f_i - dt v_ia D_a f_i + dt lambda_i sum_a d^2 f_i / dx_a^2 + (f_i^eq - f_i) / tau

  D_a     beta-mixed upwind difference by the sign of v_ia, Eqs. (SEC-VON-2a/2b)
  d^2/dx^2  central second difference (Sec. 3, after Eq. (SEC-VON-11))
  lambda_i  Eq. (SEC-VON-13): c1 dx (i = 0), c1 dx / 10 (i = 1..4), 0 (i = 5..8)

Boundaries are explicit ghost layers one cell wide (the stencil is a 5-point
cross, so no corner ghost is read). Edge kinds (Sec. 4 problem statements):
periodic; outflow (zero gradient: copy the adjacent interior cell); wall
(reflecting: mirror cell with velocities reflected); inflow (Dirichlet:
f_eq of a fixed state); shock (f_eq of state a behind, state b ahead of a
moving straight shock). Initialisation sets f = f_eq of the given fields (Sec. 4.2).

Where v_ia = 0 the convection term v_ia D_a f_i is zero and is not evaluated.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import kt

F64 = torch.float64
EDGE_NAMES = ("x-", "x+", "y-", "y+")


@dataclass
class Edge:
    kind: str = "periodic"
    split: int = 0
    a: tuple = (1.0, 0.0, 0.0, 1.0)
    b: tuple = (1.0, 0.0, 0.0, 1.0)
    x0: float = 0.0
    angle_deg: float = 90.0
    speed: float = 0.0


@dataclass
class Problem:
    nx: int
    ny: int
    dx: float
    dt: float
    c1: float
    c2: float
    eta0: float
    gamma: float = 1.4
    tau: float = 1.0
    beta: float = 0.25
    lam: list = field(default_factory=list)
    edges: list = field(default_factory=list)

    @staticmethod
    def from_dict(d):
        lam = d.get("lam")
        if lam is None:
            lam = default_lambda(d["c1"], d["dx"])
            lam[0] *= d.get("lam0_scale", 1.0)
        edges = [Edge(e["kind"], int(e.get("split", 0)), tuple(e.get("a", (1, 0, 0, 1))),
                      tuple(e.get("b", (1, 0, 0, 1))), float(e.get("x0", 0.0)),
                      float(e.get("angle_deg", 90.0)), float(e.get("speed", 0.0)))
                 for e in d["edges"]]
        return Problem(int(d["nx"]), int(d["ny"]), float(d["dx"]), float(d["dt"]), float(d["c1"]),
                       float(d["c2"]), float(d["eta0"]), float(d.get("gamma", 1.4)),
                       float(d.get("tau", 1.0)), float(d.get("beta", 0.25)), list(lam), edges)


def default_lambda(c1: float, dx: float):
    """Eq. (SEC-VON-13)."""
    return [c1 * dx] + [c1 * dx / 10.0] * 4 + [0.0] * 4


def feq_state(pb: Problem, state):
    """f_eq (9,) of a uniform state (rho, ux, uy, p), T = p / rho (P = rho R T, R = 1)."""
    r, u, v, p = (torch.tensor(float(s), dtype=F64) for s in state)
    return kt.feq(r, u, v, p / r, pb.c1, pb.c2, pb.eta0, pb.gamma)


def init(pb: Problem, rho, ux, uy, p):
    """f^0 = f_eq(rho, u, p/rho) from (ny, nx) fields."""
    rho, ux, uy, p = (a.to(F64) if isinstance(a, torch.Tensor) else torch.tensor(np.array(a, dtype=np.float64))
                      for a in (rho, ux, uy, p))
    return kt.feq(rho, ux, uy, p / rho, pb.c1, pb.c2, pb.eta0, pb.gamma)


def _ghost_line(pb: Problem, f, name: str, t: float):
    """Ghost values (9, n) along one edge, ordered along the edge."""
    e = pb.edges[EDGE_NAMES.index(name)]
    nx, ny, dx = pb.nx, pb.ny, pb.dx
    if name == "x-":
        inner, opp, axis, n = f[:, :, 0], f[:, :, nx - 1], 0, ny
    elif name == "x+":
        inner, opp, axis, n = f[:, :, nx - 1], f[:, :, 0], 0, ny
    elif name == "y-":
        inner, opp, axis, n = f[:, 0, :], f[:, ny - 1, :], 1, nx
    else:
        inner, opp, axis, n = f[:, ny - 1, :], f[:, 0, :], 1, nx
    if e.kind == "periodic":
        g = opp.clone()
    elif e.kind == "outflow":
        g = inner.clone()
    elif e.kind == "wall":
        g = inner[kt.mirror_permutation(pb.c1, pb.c2, axis)].clone()
    elif e.kind == "inflow":
        g = feq_state(pb, e.a)[:, None].expand(9, n).clone()
    elif e.kind == "shock":
        if axis != 1:
            raise ValueError("a shock edge must be a y edge")
        yg = (-0.5 if name == "y-" else ny + 0.5) * dx
        fa, fb = feq_state(pb, e.a), feq_state(pb, e.b)
        ang = math.radians(e.angle_deg)
        xs = e.x0 + yg / math.tan(ang) + e.speed * t / math.sin(ang)
        cols = []
        for i in range(n):
            xc = (i + 0.5) * dx
            cols.append(fa if xc < xs else fb)
        g = torch.stack(cols, 1)
    else:
        raise ValueError("unknown edge kind " + e.kind)
    if e.split > 0:
        g = g.clone()
        g[:, :e.split] = feq_state(pb, e.a)[:, None]
    return g


def pad(pb: Problem, f, t: float):
    """(9, ny+2, nx+2) array: interior f plus one ghost layer (corners unused, zero)."""
    ny, nx = pb.ny, pb.nx
    F = torch.zeros(9, ny + 2, nx + 2, dtype=f.dtype)
    F[:, 1:-1, 1:-1] = f
    F[:, 1:-1, 0] = _ghost_line(pb, f, "x-", t)
    F[:, 1:-1, nx + 1] = _ghost_line(pb, f, "x+", t)
    F[:, 0, 1:-1] = _ghost_line(pb, f, "y-", t)
    F[:, ny + 1, 1:-1] = _ghost_line(pb, f, "y+", t)
    return F


def upwind_derivative(fp, f0, fm, v, beta, dx):
    """Eq. (SEC-VON-2a) for v >= 0, Eq. (SEC-VON-2b) for v < 0."""
    if v >= 0:
        return (beta * fp + (1.0 - 2.0 * beta) * f0 - (1.0 - beta) * fm) / dx
    return ((1.0 - beta) * fp - (1.0 - 2.0 * beta) * f0 - beta * fm) / dx


def step(pb: Problem, f, n: int = 0):
    """f^{n+1} from f^n (shape (9, ny, nx)); n sets t = n dt for moving-shock edges."""
    return step_rows(pb, f, n, None)


def step_rows(pb: Problem, f, n: int, rows):
    """Rows `rows` (a list of y indices, None = all) of f^{n+1}; shape (9, len(rows), nx)."""
    F = pad(pb, f, n * pb.dt)
    r = torch.arange(pb.ny) if rows is None else torch.as_tensor(rows, dtype=torch.long)
    v = kt.velocities(pb.c1, pb.c2)
    rho, ux, uy, T = kt.moments(f[:, r], pb.c1, pb.c2, pb.eta0, pb.gamma)
    fe = kt.feq(rho, ux, uy, T, pb.c1, pb.c2, pb.eta0, pb.gamma)
    c = F[:, r + 1, 1:-1]
    xp, xm = F[:, r + 1, 2:], F[:, r + 1, :-2]
    yp, ym = F[:, r + 2, 1:-1], F[:, r, 1:-1]
    dx, dt = pb.dx, pb.dt
    out = []
    for i in range(9):
        vx, vy = float(v[i, 0]), float(v[i, 1])
        conv = torch.zeros_like(c[i])
        if vx != 0.0:
            conv = conv + vx * upwind_derivative(xp[i], c[i], xm[i], vx, pb.beta, dx)
        if vy != 0.0:
            conv = conv + vy * upwind_derivative(yp[i], c[i], ym[i], vy, pb.beta, dx)
        lap = (xp[i] - 2.0 * c[i] + xm[i]) / dx ** 2 + (yp[i] - 2.0 * c[i] + ym[i]) / dx ** 2
        out.append(c[i] - dt * conv + dt * pb.lam[i] * lap + (fe[i] - c[i]) / pb.tau)
    return torch.stack(out)


def store(f, storage=None):
    """f as held in memory between steps: unchanged for float64 storage; for float32
    storage each value rounded to the nearest float32 (and read back exactly), the
    arithmetic of every step staying in float64."""
    if storage is None or storage == torch.float64:
        return f
    return f.to(storage).to(F64)


def run(pb: Problem, f, nsteps: int, n0: int = 0, storage=None):
    """nsteps steps from f at time index n0; `storage` (None or torch.float32) rounds
    every stored state as in `store` (pass f already stored)."""
    for n in range(n0, n0 + nsteps):
        f = store(step(pb, f, n), storage)
    return f


def fields(pb: Problem, f):
    """(rho, ux, uy, T) of f."""
    return kt.moments(f, pb.c1, pb.c2, pb.eta0, pb.gamma)
