"""von Neumann amplification matrix of the scheme (oracle; test infrastructure only).

Sec. 3: a perturbation F_i exp(i k.x) of a uniform equilibrium grows by the
matrix G per step, Eqs. (SEC-VON-8), (SEC-VON-9), plus the dissipation term of
Eq. (SEC-VON-12):

  G_ij = (1 - 1/tau - sum_a (v_ia dt/dx) phi_a(i) - lambda_i sum_a (2 - 2 cos k_a dx) dt/dx^2) delta_ij
         + (1/tau) d f_i^eq / d f_j

  phi_a = beta e^{i k dx} + (1 - 2 beta) - (1 - beta) e^{-i k dx}      (v_ia >= 0)
        = (1 - beta) e^{i k dx} - (1 - 2 beta) - beta e^{-i k dx}      (v_ia < 0)

Readings: the "-1" of Eq. (SEC-VON-4) is -delta_ij; Eq. (SEC-VON-12) is printed
for tau = 1 and is the tau = 1 case of the form above. The Jacobian
d f^eq / d f is taken by automatic differentiation of f_eq(moments(f)).
"""
from __future__ import annotations

import cmath
import math

import torch

from . import kt

F64 = torch.float64


def collision_jacobian(rho, ux, uy, T, c1, c2, eta0, gamma):
    """J_ij = d f_i^eq / d f_j at the equilibrium of (rho, u, T); (9, 9) float64."""
    f0 = kt.feq(torch.tensor(rho, dtype=F64), torch.tensor(ux, dtype=F64),
                torch.tensor(uy, dtype=F64), torch.tensor(T, dtype=F64), c1, c2, eta0, gamma)

    def h(f):
        r, u, v, t = kt.moments(f, c1, c2, eta0, gamma)
        return kt.feq(r, u, v, t, c1, c2, eta0, gamma)

    return torch.autograd.functional.jacobian(h, f0)


def phi(v: float, kdx: float, beta: float) -> complex:
    """Eq. (SEC-VON-9)."""
    ep, em = cmath.exp(1j * kdx), cmath.exp(-1j * kdx)
    if v >= 0:
        return beta * ep + (1.0 - 2.0 * beta) - (1.0 - beta) * em
    return (1.0 - beta) * ep - (1.0 - 2.0 * beta) - beta * em


def amplification(state, params, kdx: float, kdy: float, J=None):
    """G(k) as a (9, 9) complex128 tensor.

    state = (rho, ux, uy, T); params: dict with c1, c2, eta0, gamma, tau, beta,
    dt, dx and lam (9 values).
    """
    c1, c2, eta0, gamma = params["c1"], params["c2"], params["eta0"], params["gamma"]
    tau, beta, dt, dx, lam = params["tau"], params["beta"], params["dt"], params["dx"], params["lam"]
    if J is None:
        J = collision_jacobian(*state, c1, c2, eta0, gamma)
    v = kt.velocities(c1, c2)
    G = (J / tau).to(torch.complex128)
    for i in range(9):
        vx, vy = float(v[i, 0]), float(v[i, 1])
        conv = vx * dt / dx * phi(vx, kdx, beta) + vy * dt / dx * phi(vy, kdy, beta)
        diss = lam[i] * ((2 - 2 * math.cos(kdx)) + (2 - 2 * math.cos(kdy))) * dt / dx ** 2
        G[i, i] += 1.0 - 1.0 / tau - conv - diss
    return G


def max_modulus(state, params, kdx, kdy, J=None) -> float:
    G = amplification(state, params, kdx, kdy, J)
    return float(torch.linalg.eigvals(G).abs().max())


def amplification_many(state, params, kdx, kdy, J=None):
    """G(k) of `amplification` for a list of wave vectors at once: (n, 9, 9) complex128.

    The same formula with the Eq. (SEC-VON-9) factors and the dissipation term
    evaluated per wave vector as tensors (kdx, kdy: sequences of k dx, k dy)."""
    c1, c2, eta0, gamma = params["c1"], params["c2"], params["eta0"], params["gamma"]
    tau, beta, dt, dx, lam = params["tau"], params["beta"], params["dt"], params["dx"], params["lam"]
    if J is None:
        J = collision_jacobian(*state, c1, c2, eta0, gamma)
    kx = torch.as_tensor(kdx, dtype=F64)
    ky = torch.as_tensor(kdy, dtype=F64)
    n = kx.numel()
    v = kt.velocities(c1, c2)

    def phis(vc, k):
        ep, em = torch.exp(1j * k), torch.exp(-1j * k)
        if vc >= 0:
            return beta * ep + (1.0 - 2.0 * beta) - (1.0 - beta) * em
        return (1.0 - beta) * ep - (1.0 - 2.0 * beta) - beta * em

    G = (J / tau).to(torch.complex128).expand(n, 9, 9).clone()
    for i in range(9):
        vx, vy = float(v[i, 0]), float(v[i, 1])
        conv = vx * dt / dx * phis(vx, kx) + vy * dt / dx * phis(vy, ky)
        diss = lam[i] * ((2 - 2 * torch.cos(kx)) + (2 - 2 * torch.cos(ky))) * dt / dx ** 2
        G[:, i, i] += 1.0 - 1.0 / tau - conv - diss
    return G


def max_modulus_many(state, params, kdx, kdy, J=None) -> float:
    """max over the wave vectors of the spectral radius of G(k)."""
    G = amplification_many(state, params, kdx, kdy, J)
    return float(torch.linalg.eigvals(G).abs().max())


def scan_diagonal(state, params, npts: int = 31):
    """max|omega| over k = (k, k), k dx in {0, pi/30, ..., pi} (the k grid of Sec. 3)."""
    J = collision_jacobian(*state, params["c1"], params["c2"], params["eta0"], params["gamma"])
    ks = [math.pi * m / (npts - 1) for m in range(npts)]
    return ks, [max_modulus(state, params, k, k, J) for k in ks]


def scan_modes(state, params, nx: int, ny: int):
    """Spectral radius over every Fourier mode of an nx-by-ny periodic grid."""
    J = collision_jacobian(*state, params["c1"], params["c2"], params["eta0"], params["gamma"])
    best = 0.0
    for p in range(nx):
        for q in range(ny):
            best = max(best, max_modulus(state, params, 2 * math.pi * p / nx, 2 * math.pi * q / ny, J))
    return best


def figure_params(c1=10.0, c2=20.0, eta0=10.0, alpha=0.3, dx=1.0, beta=0.25, tau=1.0,
                  dissipation=True, gamma=1.4):
    """Parameter set of the Sec. 3 figures: dt = alpha dx / c2, lambda per Eq. (SEC-VON-13)."""
    lam = [c1 * dx] + [c1 * dx / 10.0] * 4 + [0.0] * 4 if dissipation else [0.0] * 9
    return {"c1": c1, "c2": c2, "eta0": eta0, "gamma": gamma, "tau": tau, "beta": beta,
            "dt": alpha * dx / c2, "dx": dx, "lam": lam}
