"""von Neumann stability scan of the step (Sec. 3) on the GPU: binding of
lb_vn_scan and lb_vn_max_stable_dt.

A case is a uniform equilibrium state (rho, ux, uy, T) plus the scheme
parameters of a Grid; the library forms the 9x9 amplification matrix G(k) of
the implemented step at every requested wave vector and returns its spectral
radius (all arithmetic in the HIP library).
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import api
from ._lib import LbVnCase, check, lib


def case(grid: api.Grid, state, dt=None) -> LbVnCase:
    """The scan case of `grid`'s parameters at state = (rho, ux, uy, T); dt
    overrides grid.dt."""
    c = LbVnCase()
    c.rho, c.ux, c.uy, c.T = (float(v) for v in state)
    c.c1, c.c2, c.eta0, c.gamma = grid.c1, grid.c2, grid.eta0, grid.gamma
    c.tau, c.beta, c.dx = grid.tau, grid.beta, grid.dx
    c.dt = grid.dt if dt is None else float(dt)
    for i, v in enumerate(grid.lam_values()):
        c.lam[i] = v
    return c


def _cases(cases):
    arr = (LbVnCase * len(cases))(*cases)
    return arr, len(cases)


def _kvec(kdx, kdy):
    if kdx.dtype != torch.float64 or kdy.dtype != torch.float64 or kdx.shape != kdy.shape or kdx.dim() != 1 \
            or kdx.device.type != "cuda" or kdy.device != kdx.device:
        raise ValueError("kdx and kdy must be 1-D float64 GPU tensors of one length")
    return kdx.contiguous(), kdy.contiguous()


def modes(nx: int, ny: int, device="cuda"):
    """(kdx, kdy) of every Fourier mode of an nx-by-ny periodic grid: 2 pi (p/nx, q/ny)."""
    p = torch.arange(nx, dtype=torch.float64, device=device) * (2.0 * math.pi / nx)
    q = torch.arange(ny, dtype=torch.float64, device=device) * (2.0 * math.pi / ny)
    kx, ky = torch.meshgrid(p, q, indexing="ij")
    return kx.reshape(-1).contiguous(), ky.reshape(-1).contiguous()


def diagonal(npts: int = 31, device="cuda"):
    """k = (k, k) with k dx in {0, pi/(npts-1), ..., pi}: the wave vectors of the Sec. 3 figures."""
    k = torch.arange(npts, dtype=torch.float64, device=device) * (math.pi / (npts - 1))
    return k.clone(), k.clone()


def scan(cases, kdx, kdy, reduce=False):
    """Spectral radius per (case, k) as a (ncases, nk) tensor, or per case (max over k)."""
    kdx, kdy = _kvec(kdx, kdy)
    arr, n = _cases(cases)
    nk = kdx.numel()
    out = torch.empty(n if reduce else n * nk, dtype=torch.float64, device=kdx.device)
    check(lib().lb_vn_scan(arr, n, api._ptr(kdx), api._ptr(kdy), nk, 1 if reduce else 0, api._ptr(out),
                           api._stream(kdx.device)))
    return out if reduce else out.view(n, nk)


def max_stable_dt(cases, dts, kdx, kdy, tol=1e-12):
    """Per case, the largest candidate time step with every smaller candidate also
    linearly stable over the wave vectors (spectral radius <= 1 + tol); 0 if the
    first is not. dts: one ascending list for all cases, or one list per case."""
    kdx, kdy = _kvec(kdx, kdy)
    arr, n = _cases(cases)
    rows = [list(r) for r in dts] if dts and isinstance(dts[0], (list, tuple)) else [list(dts)] * n
    if len(rows) != n or len({len(r) for r in rows}) != 1:
        raise ValueError("dts needs one list, or one list per case, all of one length")
    ndt = len(rows[0])
    d = (ctypes.c_double * (n * ndt))(*[float(v) for r in rows for v in r])
    out = (ctypes.c_double * n)()
    check(lib().lb_vn_max_stable_dt(arr, n, d, ndt, api._ptr(kdx), api._ptr(kdy), kdx.numel(), float(tol),
                                    out, api._stream(kdx.device)))
    return [out[i] for i in range(n)]
