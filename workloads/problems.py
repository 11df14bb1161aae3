"""Seeded synthetic workloads: grids, parameters, boundary edges, initial fields.

A workload is a plain dict (no arithmetic of the lattice Boltzmann method is
done here); the CPU oracle and the GPU binding each turn it into their own
parameter structures. Keys:

  nx, ny          interior sites; site (i, j) has centre ((i+.5)dx, (j+.5)dx)
  dx, dt          grid spacing (dx = dy, Sec. 3 before Eq. (SEC-VON-13)) and time step
  c1, c2, eta0    KT velocity-set constants, Eqs. (e14)-(e15)
  gamma           specific-heat ratio, b = 2/(gamma-1)
  tau             relaxation time in units of dt (the paper fixes dt = Knudsen number)
  beta            upwind mixing of Eqs. (SEC-VON-2a/2b)
  lam             None for the paper's rule Eq. (SEC-VON-13), else 9 explicit values
  lam0_scale      multiplier on lambda_0 when lam is None (Fig. 9b sweep)
  edges           [x-, x+, y-, y+] edge dicts:
                    {"kind": "periodic"|"outflow"|"wall"|"inflow"|"shock",
                     "split": k, "a": state, "b": state, "x0":, "angle_deg":, "speed":}
                  "split" k > 0 makes the first k cells along the edge inflow of
                  state "a" (the double-Mach-reflection bottom edge ahead of the wall);
                  "shock": ghost cells with x < x0 + y/tan(angle) + speed*t/sin(angle)
                  take state "a", the others state "b" (moving oblique shock).
  steps           number of time steps of the workload
States are (rho, ux, uy, p) tuples.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import gasdyn

GAMMA = 1.4


def _edge(kind, **kw):
    d = {"kind": kind, "split": 0, "a": (1.0, 0.0, 0.0, 1.0), "b": (1.0, 0.0, 0.0, 1.0),
         "x0": 0.0, "angle_deg": 90.0, "speed": 0.0}
    d.update(kw)
    return d


def _base(nx, ny, dx, dt, c1, c2, eta0, steps, edges, **kw):
    d = {"nx": nx, "ny": ny, "dx": dx, "dt": dt, "c1": c1, "c2": c2, "eta0": eta0,
         "gamma": GAMMA, "tau": 1.0, "beta": 0.25, "lam": None, "lam0_scale": 1.0,
         "edges": edges, "steps": steps}
    d.update(kw)
    return d


def riemann_edges():
    """Zero-gradient x ends, periodic y: a 1D Riemann problem on a 2D grid."""
    return [_edge("outflow"), _edge("outflow"), _edge("periodic"), _edge("periodic")]


def riemann_fields(cfg, left, right, x_disc):
    """(rho, ux, uy, p) arrays of shape (ny, nx): left state for x < x_disc."""
    nx, ny, dx = cfg["nx"], cfg["ny"], cfg["dx"]
    x = (np.arange(nx) + 0.5) * dx
    out = []
    for k in range(4):
        row = np.where(x < x_disc, left[k], right[k]).astype(np.float64)
        out.append(np.ascontiguousarray(np.broadcast_to(row, (ny, nx))))
    return tuple(out)


# ------------------------------------------------------------------ configurations

def sod(nx=200, ny=4, steps=500):
    """Sod shock tube: (1,0,0,1) | (0.125,0,0,0.1) on [0,1]; c1,c2,eta0 = 1,3,2."""
    dx = 1.0 / nx
    cfg = _base(nx, ny, dx, 0.08 * dx, 1.0, 3.0, 2.0, steps, riemann_edges(), name="sod")
    cfg["left"], cfg["right"], cfg["x_disc"] = (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1), 0.5
    return cfg


def ratio1000(nx=2000, ny=4, steps=4000):
    """1000:1 Riemann problem, Eq. (Riemann-2); dx = 0.0025, c1,c2,eta0 = 3,9,5.

    dt = 0.072 dx/c2 = 2e-5 (the printed 2e-4 is not stable, see the design notes)."""
    dx = 0.0025
    cfg = _base(nx, ny, dx, 2e-5, 3.0, 9.0, 5.0, steps, riemann_edges(), name="ratio1000")
    cfg["left"], cfg["right"], cfg["x_disc"] = (1000.0, 0.0, 0.0, 1000.0), (1.0, 0.0, 0.0, 1.0), 0.5 * nx * dx
    return cfg


def mach30(nx=1200, ny=4, steps=None, alpha=0.05, beta=0.25, lam0_scale=1.0):
    """Mach-30 Riemann problem, Eq. (Riemann-1); dx = 0.01, c1,c2,eta0 = 25,50,30."""
    dx = 0.01
    dt = alpha * dx / 50.0
    if steps is None:
        steps = int(round(0.36 / dt))
    cfg = _base(nx, ny, dx, dt, 25.0, 50.0, 30.0, steps, riemann_edges(), name="mach30",
                beta=beta, lam0_scale=lam0_scale)
    cfg["left"], cfg["right"], cfg["x_disc"] = (1.4, 30.0, 0.0, 1.0), (1.4, 0.0, 0.0, 1.0), 0.25 * nx * dx
    return cfg


def regular_reflection_paper(alpha=0.3, t_end=2.5, seed=0):
    """The regular reflection at the paper's resolution (Sec. 4.2, Fig. 11): 900 x 300
    cells of 0.01 (9 x 3), Mach-10 inflow (1, 10, 0, 1/1.4), 30-degree incident shock
    (top state from the oblique-shock relations, which give the printed
    (5, 8, -3.4641, 20.7143)), c1,c2,eta0 = 10,20,15, run to t = t_end. The printed
    dt = 1.5e-4 is alpha = c2 dt/dx = 0.3."""
    dt = alpha * 0.01 / 20.0
    return regular_reflection(nx=900, ny=300, steps=int(round(t_end / dt)), mach=10.0, seed=seed,
                              c=(10.0, 20.0, 15.0), alpha=alpha)


def init_riemann(cfg):
    return riemann_fields(cfg, cfg["left"], cfg["right"], cfg["x_disc"])


def regular_reflection(nx=300, ny=90, steps=20000, mach=2.9, wave_angle_deg=30.0, seed=0, c=(3.0, 9.0, 5.0),
                       alpha=0.2):
    """Regular reflection of an oblique shock off the bottom wall (Sec. 4.2).

    Left: inflow (1, mach, 0, 1/gamma) (sound speed 1); top: the state behind a
    `wave_angle_deg` oblique shock of that inflow; bottom: reflecting wall;
    right: supersonic outflow. c1,c2,eta0 = c (3,9,5 by default); dt = alpha dx/c2.
    """
    dx = 0.01
    inflow = (1.0, mach, 0.0, 1.0 / GAMMA)
    top = gasdyn.oblique_shock_state(GAMMA, inflow, wave_angle_deg)
    edges = [_edge("inflow", a=inflow), _edge("outflow"), _edge("wall"), _edge("inflow", a=top)]
    cfg = _base(nx, ny, dx, alpha * dx / c[1], c[0], c[1], c[2], steps, edges, name="regular_reflection")
    cfg["inflow"], cfg["top"], cfg["seed"] = inflow, top, seed
    cfg["wave_angle_deg"] = wave_angle_deg
    return cfg


def init_regular_reflection(cfg):
    """Inflow state everywhere (Sec. 4.2), density times (1 + U[-1e-6, 1e-6])."""
    nx, ny = cfg["nx"], cfg["ny"]
    rng = np.random.default_rng(cfg["seed"])
    xi = rng.uniform(-1e-6, 1e-6, size=(ny, nx))
    r, u, v, p = cfg["inflow"]
    return (r * (1.0 + xi), np.full((ny, nx), u), np.full((ny, nx), v), np.full((ny, nx), p))


def double_mach(nx=960, ny=240, steps=2000, length=9.6, wall_cells=None, alpha=0.025, c=(8.0, 16.0, 10.0)):
    """Double Mach reflection (Sec. 4.2, Fig. 12): Mach-10 shock at 60 deg to the wall.

    Pre-shock (1.4, 0, 0, 1); post-shock from the normal-shock relations; the
    wall starts `wall_cells` cells from the lower-left corner (20 at dx = 0.01,
    the same physical offset 0.2 at other resolutions); c1,c2,eta0 = c (8,16,10 printed);
    dt = alpha dx/c2 with alpha = 0.025 (larger alpha lets the reflected shock
    foot at the wall drive T negative: the oracle blows up near step 600 at
    alpha = 0.1 and near step 1500 at alpha = 0.05).
    """
    dx = length / nx
    x0 = 0.2 if wall_cells is None else wall_cells * dx
    split = int(round(x0 / dx))
    pre = (1.4, 0.0, 0.0, 1.0)
    post = gasdyn.moving_shock_post_state(GAMMA, (1.4, 1.0), 10.0, -30.0)
    edges = [_edge("inflow", a=post), _edge("outflow"),
             _edge("wall", split=split, a=post),
             _edge("shock", a=post, b=pre, x0=x0, angle_deg=60.0, speed=10.0)]
    cfg = _base(nx, ny, dx, alpha * dx / c[1], c[0], c[1], c[2], steps, edges, name="double_mach")
    cfg["pre"], cfg["post"], cfg["x0"] = pre, post, x0
    return cfg


def init_double_mach(cfg):
    nx, ny, dx = cfg["nx"], cfg["ny"], cfg["dx"]
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    behind = X < cfg["x0"] + Y / math.tan(math.radians(60.0))
    out = []
    for k in range(4):
        out.append(np.where(behind, cfg["post"][k], cfg["pre"][k]).astype(np.float64))
    return tuple(out)


def roofline_grid(nx=8192, ny=2048):
    """The double-Mach-reflection field on a grid too large for the on-chip caches."""
    cfg = double_mach(nx=nx, ny=ny, length=9.6)
    cfg["workload"] = "double-Mach-reflection field on %dx%d" % (nx, ny)
    return cfg


def dmr_target_density(cfg, rho0, seed=1):
    """Target initial density: pre-shock sites times (1 + 0.01 U[-1,1])."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=rho0.shape)
    pre = np.isclose(rho0, cfg["pre"][0])
    return np.where(pre, rho0 * (1.0 + 0.01 * xi), rho0)


def init_fields(cfg):
    name = cfg["name"]
    if name in ("sod", "ratio1000", "mach30", "batched"):
        return init_riemann(cfg)
    if name == "regular_reflection":
        return init_regular_reflection(cfg)
    if name == "double_mach":
        return init_double_mach(cfg)
    if name == "periodic_smooth":
        return init_periodic_smooth(cfg)
    raise KeyError(name)


# ------------------------------------------------------------------ generic test fields

def periodic_smooth(nx=24, ny=16, steps=10, seed=3, c=(3.0, 9.0, 5.0), alpha=0.1):
    """Fully periodic grid with a smooth random field (conservation tests)."""
    dx = 0.01
    edges = [_edge("periodic") for _ in range(4)]
    cfg = _base(nx, ny, dx, alpha * dx / c[1], c[0], c[1], c[2], steps, edges, name="periodic_smooth")
    cfg["seed"] = seed
    return cfg


def init_periodic_smooth(cfg):
    """Low Fourier modes with seeded amplitudes and phases; rho, p stay positive."""
    nx, ny = cfg["nx"], cfg["ny"]
    rng = np.random.default_rng(cfg["seed"])
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)
    fields = []
    base = [1.0, 0.5, -0.3, 1.0]
    amp = [0.2, 0.3, 0.3, 0.2]
    for k in range(4):
        acc = np.full((ny, nx), base[k])
        for (kx, ky) in ((1, 0), (0, 1), (1, 1), (2, 1)):
            a = rng.uniform(-1, 1) * amp[k] / 2
            ph = rng.uniform(0, 2 * math.pi)
            acc = acc + a * np.cos(2 * math.pi * (kx * X + ky * Y) + ph)
        fields.append(acc)
    return tuple(fields)


def random_distributions(nx, ny, seed, lo=0.5, hi=1.5):
    """A raw (9, ny, nx) array of positive values: a non-equilibrium input state."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(9, ny, nx))


# ------------------------------------------------------------------ batched draws

SCREEN_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batched_screen.json")


def batched_params(left, right, star):
    """Per-problem constants from the paper's guidance (end of Sec. 3): c1 about the
    largest flow speed (here at least the largest thermal speed sqrt(T) too), c2 = 3 c1,
    eta0 between c1 and c2 (2 c1). Speeds and temperatures include the exact star states."""
    U = max(abs(left[1]), abs(right[1]), abs(star.u))
    Tmax = max(left[2] / left[0], right[2] / right[0], star.p / star.rho_l, star.p / star.rho_r)
    c1 = max(U, math.sqrt(Tmax))
    return c1, 3.0 * c1, 2.0 * c1


def batched_candidate(seed, slot, attempt_rng, lmin=128, lmax=8192):
    """One candidate draw for output slot `slot` from that slot's generator.

    rho and p log-uniform in [0.1, 1000] per side, redrawn until max/min <= 1000 for
    both; |u| = M c_side with M ~ U[0, 5] (every 8th slot: U[5, 30]) and a random sign
    per side; draws that create vacuum are redrawn (counted). Returns
    (L, left, right, star, fast, vacuum_redraws).
    """
    rng = attempt_rng
    L = int(round(math.exp(rng.uniform(math.log(lmin), math.log(lmax)))))
    fast = (slot % 8 == 7)
    vac = 0
    while True:
        while True:
            rho = np.exp(rng.uniform(math.log(0.1), math.log(1000.0), size=2))
            pr = np.exp(rng.uniform(math.log(0.1), math.log(1000.0), size=2))
            if rho.max() / rho.min() <= 1000.0 and pr.max() / pr.min() <= 1000.0:
                break
        cs = np.sqrt(GAMMA * pr / rho)
        M = rng.uniform(5.0, 30.0, size=2) if fast else rng.uniform(0.0, 5.0, size=2)
        sgn = np.where(rng.uniform(size=2) < 0.5, -1.0, 1.0)
        u = sgn * M * cs
        left = (float(rho[0]), float(u[0]), float(pr[0]))
        right = (float(rho[1]), float(u[1]), float(pr[1]))
        try:
            st = gasdyn.riemann_star(GAMMA, left, right)
        except ValueError:
            vac += 1
            continue
        return L, left, right, st, fast, vac


def batched_cfg(L, left, right, star, fast, steps, alpha=0.025, ny=4):
    c1, c2, eta0 = batched_params(left, right, star)
    dx = 1.0 / L
    cfg = _base(L, ny, dx, alpha * dx / c2, c1, c2, eta0, steps, riemann_edges(), name="batched")
    cfg["left"] = (left[0], left[1], 0.0, left[2])
    cfg["right"] = (right[0], right[1], 0.0, right[2])
    cfg["x_disc"] = 0.5
    cfg["fast"] = fast
    return cfg


def screen_key(seed, steps, alpha):
    return "seed=%d steps=%d alpha=%g" % (seed, steps, alpha)


def load_screen(seed, steps, alpha):
    """Slot attempts rejected by the FP64 CPU screen (a stored list), or None."""
    try:
        with open(SCREEN_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(screen_key(seed, steps, alpha))
    if e is None:
        return None
    return {(int(a), int(b)) for a, b in e["rejected"]}


def batched(nprob=256, seed=0, steps=2000, alpha=0.025, ny=4, screen=True, max_attempts=64):
    """Independent 1D Riemann problems of uneven lengths L log-uniform in [128, 8192].

    Slot p draws from its own generator default_rng([seed, p]); an attempt that the
    stored FP64 screen rejected (the scheme leaves the physical range within `steps`
    steps: non-finite, rho <= 0 or rho > 1e6) is redrawn from the same generator.
    dx = 1/L, dt = alpha dx / c2, ny rows (periodic y, zero-gradient x).
    Returns (cfgs, info) with info = {"vacuum_redraws", "unstable_redraws", "screened", "attempts",
    "accepted_fraction"}: the workload is the seeded distribution conditioned on the oracle
    keeping the run in the physical range (about 60% of the draws for seed 0).
    """
    rejected = load_screen(seed, steps, alpha) if screen else None
    out, vac, unstable = [], 0, 0
    for p in range(nprob):
        rng = np.random.default_rng([seed, p])
        for a in range(max_attempts):
            L, left, right, st, fast, v = batched_candidate(seed, p, rng)
            vac += v
            if rejected is not None and (p, a) in rejected:
                unstable += 1
                continue
            out.append(batched_cfg(L, left, right, st, fast, steps, alpha, ny))
            break
        else:
            raise RuntimeError("slot %d: no accepted draw in %d attempts" % (p, max_attempts))
    return out, {"vacuum_redraws": vac, "unstable_redraws": unstable, "screened": rejected is not None,
                 "attempts": nprob + unstable, "accepted_fraction": nprob / (nprob + unstable)}


# ------------------------------------------------------------------ von Neumann chooser inputs (batched draws)

# Candidate alpha = c2 dt / dx, ascending, and the growth tolerance of the chooser: a
# mode may grow by at most a factor 2 over a 2000-step run (radius <= 1 + ln 2 / 2000).
VN_ALPHAS = (0.025, 0.05, 0.075, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35, 0.4, 0.45, 0.5)
VN_TOL = math.log(2.0) / 2000


def vn_wave_vectors(nkx=64):
    """(kdx, kdy) lists: nkx values of k_x dx on [0, 2 pi) times the 4 modes k_y dy of a
    4-row periodic grid (0, pi/2, pi, 3 pi/2)."""
    kx = [k * (2 * math.pi / nkx) for k in range(nkx) for _ in range(4)]
    ky = [j * (math.pi / 2) for _ in range(nkx) for j in range(4)]
    return kx, ky


def batched_vn_states(cfg):
    """The uniform states (rho, ux, uy, T) whose linear stability bounds a batched
    Riemann problem's time step: its left and right states and the two exact star
    states between them."""
    L, R = cfg["left"], cfg["right"]
    st = gasdyn.riemann_star(cfg["gamma"], (L[0], L[1], L[3]), (R[0], R[1], R[3]))
    return [(L[0], L[1], 0.0, L[3] / L[0]), (R[0], R[1], 0.0, R[3] / R[0]),
            (st.rho_l, st.u, 0.0, st.p / st.rho_l), (st.rho_r, st.u, 0.0, st.p / st.rho_r)]
