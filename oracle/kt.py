"""Kataoka-Tsutahara D2V9 discrete-velocity model (oracle; test infrastructure only).

Sec. 2 of the paper:
  velocities  Eq. (e14)   v_0 = 0; v_1..4 = c1 (cos, sin)(pi (i+1)/2);
                          v_5..8 = c2 (cos, sin)(pi ((i+1)/2 + 1/4))
  eta_i       Eq. (e15)   eta_0 = eta0, eta_1..8 = 0
  moments     Eqs. (e4), (e5), (e7)   rho = sum f, rho u = sum f v,
                          rho (b T + u^2) = sum f (v^2 + eta^2), R = 1, b = 2/(gamma-1)
  equilibrium Eqs. (e16)-(e18)  f_eq = rho (A + B (v.u) + D (v.u)^2)

Readings of garbled formulas (both forced by the moment constraints (e4)-(e8),
which fail with the printed forms):
  * the diagonal group of Eq. (e14) is printed (cos, cos); read (cos, sin);
  * A_0 of Eq. (e17) is printed (b-2) T / eta0; read (b-2) T / eta0^2.
"""
from __future__ import annotations

import math

import mpmath
import torch

F64 = torch.float64


def velocities(c1: float, c2: float) -> torch.Tensor:
    """(9, 2) discrete velocities of Eq. (e14), diagonal group read as (cos, sin).

    Each component c cos(theta), c sin(theta) is evaluated in 40-digit
    arithmetic and rounded once to float64, so the set keeps its exact
    symmetries (|v_x| = |v_y| on the diagonals, zeros exactly zero); float64
    trig of the large angles pi (i+1)/2 would be off by several ulps.
    """
    with mpmath.workdps(40):
        v = torch.zeros(9, 2, dtype=F64)
        for i in range(1, 5):
            th = mpmath.pi * mpmath.mpf(i + 1) / 2
            v[i, 0], v[i, 1] = float(c1 * mpmath.cos(th)), float(c1 * mpmath.sin(th))
        for i in range(5, 9):
            th = mpmath.pi * (mpmath.mpf(i + 1) / 2 + mpmath.mpf(1) / 4)
            v[i, 0], v[i, 1] = float(c2 * mpmath.cos(th)), float(c2 * mpmath.sin(th))
    v[v.abs() < 1e-30 * max(c1, c2)] = 0.0
    return v


def energy_weights(c1: float, c2: float, eta0: float) -> torch.Tensor:
    """|v_i|^2 + eta_i^2 of Eq. (e7): eta0^2, c1^2 (i = 1..4), c2^2 (i = 5..8).

    |v_i| is c1 or c2 by Eq. (e14); the squares are rounded once, not rebuilt
    from rounded components.
    """
    return torch.tensor([eta0 * eta0] + [c1 * c1] * 4 + [c2 * c2] * 4, dtype=F64)


def etas(eta0: float) -> torch.Tensor:
    """Eq. (e15)."""
    e = torch.zeros(9, dtype=F64)
    e[0] = eta0
    return e


def b_of_gamma(gamma: float) -> float:
    """b = 2/(gamma - 1) (Sec. 2, after Eq. (e2))."""
    return 2.0 / (gamma - 1.0)


def coefficients(T, usq, c1, c2, eta0, b):
    """A_i, B_i, D_i of Eqs. (e17)-(e18) as lists of 9 tensors (or floats).

    `T` and `usq` (= u_alpha u_alpha) are broadcastable tensors.
    """
    c1s, c2s, e2 = c1 * c1, c2 * c2, eta0 * eta0
    A0 = (b - 2.0) * T / e2
    A1 = (-c2s + ((b - 2.0) * c2s / e2 + 2.0) * T + (c2s / c1s) * usq) / (4.0 * (c1s - c2s))
    A5 = (-c1s + ((b - 2.0) * c1s / e2 + 2.0) * T + (c1s / c2s) * usq) / (4.0 * (c2s - c1s))
    B1 = (-c2s + (b + 2.0) * T + usq) / (2.0 * c1s * (c1s - c2s))
    B5 = (-c1s + (b + 2.0) * T + usq) / (2.0 * c2s * (c2s - c1s))
    D1 = 1.0 / (2.0 * c1s * c1s)
    D5 = 1.0 / (2.0 * c2s * c2s)
    A = [A0] + [A1] * 4 + [A5] * 4
    B = [0.0] + [B1] * 4 + [B5] * 4
    D = [0.0] + [D1] * 4 + [D5] * 4
    return A, B, D


def feq(rho, ux, uy, T, c1, c2, eta0, gamma):
    """Equilibrium distributions, Eq. (e16): returns a (9, *rho.shape) tensor."""
    b = b_of_gamma(gamma)
    v = velocities(c1, c2)
    usq = ux * ux + uy * uy
    A, B, D = coefficients(T, usq, c1, c2, eta0, b)
    out = []
    for i in range(9):
        vu = v[i, 0] * ux + v[i, 1] * uy
        out.append(rho * (A[i] + B[i] * vu + D[i] * vu * vu))
    return torch.stack(out)


def moments(f, c1, c2, eta0, gamma):
    """(rho, ux, uy, T) from distributions f of shape (9, ...), Eqs. (e4), (e5), (e7)."""
    b = b_of_gamma(gamma)
    v = velocities(c1, c2)
    et = etas(eta0)
    shape = (9,) + (1,) * (f.dim() - 1)
    rho = f.sum(0)
    jx = (f * v[:, 0].reshape(shape)).sum(0)
    jy = (f * v[:, 1].reshape(shape)).sum(0)
    w = energy_weights(c1, c2, eta0).reshape(shape)
    E = (f * w).sum(0)
    ux = jx / rho
    uy = jy / rho
    T = (E / rho - ux * ux - uy * uy) / b
    return rho, ux, uy, T


def conserved(f, c1, c2, eta0):
    """Column sums sum_i psi_i f_i for psi = 1, v_x, v_y, v^2 + eta^2 (mass, momentum, energy)."""
    v = velocities(c1, c2)
    et = etas(eta0)
    shape = (9,) + (1,) * (f.dim() - 1)
    return (f.sum(0), (f * v[:, 0].reshape(shape)).sum(0), (f * v[:, 1].reshape(shape)).sum(0),
            (f * energy_weights(c1, c2, eta0).reshape(shape)).sum(0))


def mirror_permutation(c1: float, c2: float, axis: int):
    """Index map i -> j with v_j equal to v_i reflected across a wall normal to `axis`."""
    v = velocities(c1, c2)
    perm = []
    for i in range(9):
        w = v[i].clone()
        w[axis] = -w[axis]
        j = int(torch.argmin(((v - w) ** 2).sum(1)))
        perm.append(j)
    return perm
