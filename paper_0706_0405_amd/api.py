"""Python binding of the lbkt C ABI over torch device tensors.

Every function marshals arguments and calls the HIP library; all arithmetic of
the step runs in the library's kernels. Distribution arrays are torch tensors
of shape (9, ny, pitch) (float64 for LB_F64, float32 for LB_F32); macroscopic
fields are contiguous (ny, nx) float64 tensors. Work is enqueued on torch's
current stream of the tensors' device.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import LB_F32, LB_F64, LbEdge, LbGrid, LbState, LbTile, check, lib

PREC = {"f64": LB_F64, "f32": LB_F32, LB_F64: LB_F64, LB_F32: LB_F32}
DTYPE = {LB_F64: torch.float64, LB_F32: torch.float32}


def _prec(p):
    return PREC[p]


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class Grid:
    """A grid and its scheme parameters (the fields of lb_grid)."""
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
    lam: list | None = None          # None: Eq. (SEC-VON-13) via lb_default_lambda
    lam0_scale: float = 1.0
    edges: list = field(default_factory=list)

    @staticmethod
    def from_workload(d):
        return Grid(int(d["nx"]), int(d["ny"]), float(d["dx"]), float(d["dt"]), float(d["c1"]), float(d["c2"]),
                    float(d["eta0"]), float(d.get("gamma", 1.4)), float(d.get("tau", 1.0)),
                    float(d.get("beta", 0.25)), d.get("lam"), float(d.get("lam0_scale", 1.0)),
                    [dict(e) for e in d["edges"]])

    @property
    def pitch(self):
        return (self.nx + 63) // 64 * 64

    def c(self) -> LbGrid:
        g = LbGrid()
        g.nx, g.ny, g.pitch = self.nx, self.ny, self.pitch
        g.dx, g.dt, g.c1, g.c2, g.eta0 = self.dx, self.dt, self.c1, self.c2, self.eta0
        g.gamma, g.tau, g.beta = self.gamma, self.tau, self.beta
        if self.lam is None:
            check(lib().lb_default_lambda(ctypes.byref(g)))
            g.lam[0] = g.lam[0] * self.lam0_scale
        else:
            for i in range(9):
                g.lam[i] = float(self.lam[i])
        for k, e in enumerate(self.edges):
            E = LbEdge()
            E.kind = _lib.BC[e["kind"]]
            E.split = int(e.get("split", 0))
            E.a = LbState(*[float(v) for v in e.get("a", (1.0, 0.0, 0.0, 1.0))])
            E.b = LbState(*[float(v) for v in e.get("b", (1.0, 0.0, 0.0, 1.0))])
            E.x0 = float(e.get("x0", 0.0))
            E.angle_deg = float(e.get("angle_deg", 90.0))
            E.speed = float(e.get("speed", 0.0))
            g.edge[k] = E
        return g

    def lam_values(self):
        g = self.c()
        return [g.lam[i] for i in range(9)]


def validate(grid: Grid):
    check(lib().lb_validate(ctypes.byref(grid.c())))


def empty(grid: Grid, prec="f64", device="cuda"):
    """Uninitialised distribution array (9, ny, pitch)."""
    p = _prec(prec)
    return torch.empty((9, grid.ny, grid.pitch), dtype=DTYPE[p], device=device)


def _check_f(grid, p, f, name):
    if f.dtype != DTYPE[p] or tuple(f.shape) != (9, grid.ny, grid.pitch) or not f.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor of shape (9, %d, %d)"
                         % (name, DTYPE[p], grid.ny, grid.pitch))
    if f.device.type != "cuda":
        raise ValueError("%s must be a GPU tensor" % name)


def _check_field(grid, t, name):
    if t.dtype != torch.float64 or tuple(t.shape) != (grid.ny, grid.nx) or not t.is_contiguous() \
            or t.device.type != "cuda":
        raise ValueError("%s must be a contiguous float64 GPU tensor of shape (%d, %d)" % (name, grid.ny, grid.nx))


def init(grid: Grid, rho, ux, uy, p, prec="f64", out=None):
    """f = f_eq(rho, u, p/rho) (lb_init)."""
    pr = _prec(prec)
    for t, n in ((rho, "rho"), (ux, "ux"), (uy, "uy"), (p, "p")):
        _check_field(grid, t, n)
    f = empty(grid, pr, rho.device) if out is None else out
    _check_f(grid, pr, f, "f")
    check(lib().lb_init(ctypes.byref(grid.c()), pr, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(p), _ptr(f),
                        _stream(rho.device)))
    return f


def _tile(tile, steps=0):
    """(block_x, rows[, blocks[, steps]]) -> lb_tile; None = the library's default shape.
    steps: time steps per pass of lb_run (0 = the tile's own, else the default; 1, 2 or 3)."""
    if tile is None and not steps:
        return None
    t = tuple(tile) if tile is not None else (0, 0)
    blocks = int(t[2]) if len(t) > 2 else 0
    if not steps and len(t) > 3:   # a tuned shape carries its steps per pass
        steps = int(t[3])
    return ctypes.byref(LbTile(int(t[0]), int(t[1]), blocks, int(steps)))


def step(grid: Grid, f_in, f_out, n=0, prec="f64", tile=None):
    """f_out = S(f_in) at time index n (lb_step / lb_step_tiled)."""
    pr = _prec(prec)
    _check_f(grid, pr, f_in, "f_in")
    _check_f(grid, pr, f_out, "f_out")
    check(lib().lb_step_tiled(ctypes.byref(grid.c()), pr, _ptr(f_in), _ptr(f_out), int(n), _tile(tile),
                              _stream(f_in.device)))
    return f_out


def run(grid: Grid, f_a, f_b, nsteps, n0=0, prec="f64", use_graph=False, tile=None, steps_per_pass=0):
    """nsteps ping-pong steps; returns the tensor holding the result (lb_run).
    steps_per_pass: 1 = one step per launch, 2 = two, 3 = three (FP64 arrays); 0 = the
    library default (three on FP64 arrays below 4 GiB with ny >= 32, sixteen on 4-row grids
    with a periodic y axis and at least 64 columns, else two)."""
    pr = _prec(prec)
    _check_f(grid, pr, f_a, "f_a")
    _check_f(grid, pr, f_b, "f_b")
    check(lib().lb_run(ctypes.byref(grid.c()), pr, _ptr(f_a), _ptr(f_b), int(n0), int(nsteps),
                       1 if use_graph else 0, _tile(tile, steps_per_pass), _stream(f_a.device)))
    return f_a if nsteps % 2 == 0 else f_b


def moments(grid: Grid, f, prec="f64", flags=True, check_finite=False):
    """(rho, ux, uy, T[, flags]) as (ny, nx) float64 tensors; flags = int64 tensor (4,).
    check_finite: wait for the result and raise LbError (LB_ENONFINITE) if some site
    is non-finite or has rho <= 0 (lb_check_flags)."""
    pr = _prec(prec)
    _check_f(grid, pr, f, "f")
    dev = f.device
    outs = [torch.empty((grid.ny, grid.nx), dtype=torch.float64, device=dev) for _ in range(4)]
    fl = torch.empty(4, dtype=torch.int32, device=dev) if (flags or check_finite) else None
    check(lib().lb_moments(ctypes.byref(grid.c()), pr, _ptr(f), *[_ptr(o) for o in outs], _ptr(fl),
                           _stream(dev)))
    if check_finite:
        check_flags(fl)
    if flags:
        return (*outs, fl.to(torch.int64) & 0xFFFFFFFF)
    return tuple(outs)


def check_flags(flags):
    """Raise LbError (LB_ENONFINITE) when the raw device flags word that lb_moments
    wrote (an int32 tensor of 4) reports a non-finite site or rho <= 0; returns the
    four words as Python ints otherwise (lb_check_flags, synchronous)."""
    if flags.dtype != torch.int32 or flags.numel() != 4 or flags.device.type != "cuda":
        raise ValueError("flags must be the int32 device tensor of 4 words that lb_moments filled")
    host = (ctypes.c_uint32 * 4)()
    check(lib().lb_check_flags(_ptr(flags), host, _stream(flags.device)))
    return list(host)


def invariants(grid: Grid, f, prec="f64", out=None, noalloc=False):
    """(4,) float64 device tensor: totals of rho, rho ux, rho uy, rho (b T + u^2).
    noalloc: lb_invariants_noalloc (the library's fixed array instead of a workspace)."""
    pr = _prec(prec)
    _check_f(grid, pr, f, "f")
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=f.device)
    if out.dtype != torch.float64 or out.numel() != 4 or not out.is_contiguous() or out.device.type != "cuda":
        raise ValueError("out must be a contiguous float64 GPU tensor of 4 elements")
    fn = lib().lb_invariants_noalloc if noalloc else lib().lb_invariants
    check(fn(ctypes.byref(grid.c()), pr, _ptr(f), _ptr(out), _stream(f.device)))
    return out


def step_adjoint(grid: Grid, f_n, g_np1, g_n=None, n=0, prec="f64"):
    """g_n = (dS/df at f_n)^T g_np1 (lb_step_adjoint); g arrays are float64."""
    pr = _prec(prec)
    _check_f(grid, pr, f_n, "f_n")
    _check_f(grid, LB_F64, g_np1, "g_np1")
    if g_n is None:
        g_n = empty(grid, LB_F64, f_n.device)
    _check_f(grid, LB_F64, g_n, "g_n")
    check(lib().lb_step_adjoint(ctypes.byref(grid.c()), pr, _ptr(f_n), _ptr(g_np1), _ptr(g_n), int(n),
                                _stream(f_n.device)))
    return g_n


def run_record(grid: Grid, f0, outs, n0=0, prec="f64"):
    """outs[j] = state after step n0 + j from f0 (lb_run_record)."""
    pr = _prec(prec)
    _check_f(grid, pr, f0, "f0")
    for o in outs:
        _check_f(grid, pr, o, "out")
    arr = (ctypes.c_void_p * max(1, len(outs)))(*[o.data_ptr() for o in outs])
    check(lib().lb_run_record(ctypes.byref(grid.c()), pr, _ptr(f0), arr, int(n0), len(outs), _stream(f0.device)))
    return outs


def adjoint_run(grid: Grid, states, g, work, n0=0, prec="f64"):
    """Reverse sweep over states (f at n0 .. n0+len-1) starting from g = dL/df^(n0+len);
    returns the tensor (g or work) that holds dL/df^(n0) (lb_adjoint_run)."""
    pr = _prec(prec)
    for t in states:
        _check_f(grid, pr, t, "state")
    _check_f(grid, LB_F64, g, "g")
    _check_f(grid, LB_F64, work, "work")
    arr = (ctypes.c_void_p * max(1, len(states)))(*[t.data_ptr() for t in states])
    check(lib().lb_adjoint_run(ctypes.byref(grid.c()), pr, arr, _ptr(g), _ptr(work), int(n0), len(states),
                               _stream(g.device)))
    return g if len(states) % 2 == 0 else work


def init_adjoint(grid: Grid, rho, ux, uy, p, g_f0):
    """dL/drho0 from dL/df0 at fixed u and p (lb_init_adjoint)."""
    for t, n in ((rho, "rho"), (ux, "ux"), (uy, "uy"), (p, "p")):
        _check_field(grid, t, n)
    _check_f(grid, LB_F64, g_f0, "g_f0")
    out = torch.empty((grid.ny, grid.nx), dtype=torch.float64, device=rho.device)
    check(lib().lb_init_adjoint(ctypes.byref(grid.c()), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(p), _ptr(g_f0),
                                _ptr(out), _stream(rho.device)))
    return out


def autotune(grid: Grid, f_a, f_b, prec="f64", reps=10):
    """Fastest (block_x, rows, blocks, steps_per_pass) for lb_run on this grid and its
    time per step, timed with HIP events (lb_autotune)."""
    pr = _prec(prec)
    _check_f(grid, pr, f_a, "f_a")
    _check_f(grid, pr, f_b, "f_b")
    best = LbTile()
    ms = ctypes.c_float()
    check(lib().lb_autotune(ctypes.byref(grid.c()), pr, _ptr(f_a), _ptr(f_b), int(reps), ctypes.byref(best),
                            ctypes.byref(ms), _stream(f_a.device)))
    return (best.block_x, best.rows, best.blocks, best.steps), ms.value


def interior(grid: Grid, f):
    """View (9, ny, nx) of the interior of a distribution array."""
    return f[:, :, :grid.nx]


class Batch:
    """Independent grids advanced together (lb_batch_*): one packed array per buffer."""

    def __init__(self, grids, prec="f32"):
        self.grids = list(grids)
        self.prec = _prec(prec)
        n = len(self.grids)
        arr = (LbGrid * n)(*[g.c() for g in self.grids])
        h = ctypes.c_void_p()
        check(lib().lb_batch_create(n, arr, self.prec, ctypes.byref(h)))
        self.h = h
        offs = (ctypes.c_int64 * n)()
        pitches = (ctypes.c_int64 * n)()
        total = ctypes.c_int64()
        check(lib().lb_batch_layout(h, offs, pitches, ctypes.byref(total)))
        self.offsets = list(offs)
        self.pitches = list(pitches)
        self.total = total.value

    def empty(self, device="cuda"):
        return torch.empty(self.total, dtype=DTYPE[self.prec], device=device)

    def view(self, buf, p):
        """The (9, ny, pitch) distribution array of problem p inside a packed buffer."""
        g = self.grids[p]
        o = self.offsets[p]
        return buf[o:o + 9 * g.ny * self.pitches[p]].view(9, g.ny, self.pitches[p])

    def set_tile(self, block_x, steps_per_pass=0, persistent_blocks=0, polls=0):
        """Threads per work item (64, 128, 256) and time steps per pass (0 = default; 1, 2,
        or 4, 6, 8 for a batch of 4-row y-periodic problems, whose default is 4 in FP32 and 8 in
        FP64 storage; in FP32 storage at width 64, that batch's default width, the deep passes
        run a strip's four rows on the four wavefronts of a 256-thread block);
        persistent_blocks > 0: all two-step passes in one launch of at most that many
        co-resident blocks (polls: poll budget per wait, 0 = the library's default)."""
        check(lib().lb_batch_set_tile(self.h, ctypes.byref(LbTile(int(block_x), int(polls), int(persistent_blocks),
                                                                  int(steps_per_pass)))))

    def status(self, device=None):
        """Raise LbError if a persistent launch gave up waiting (lb_batch_status, synchronous)."""
        check(lib().lb_batch_status(self.h, _stream(device)))

    def step(self, f_a, f_b, nsteps):
        """nsteps steps of every problem in one graph launch; returns the result buffer."""
        for t in (f_a, f_b):
            if t.dtype != DTYPE[self.prec] or t.numel() != self.total or not t.is_contiguous():
                raise ValueError("batch buffers must be contiguous with %d elements" % self.total)
        check(lib().lb_step_batched(self.h, _ptr(f_a), _ptr(f_b), int(nsteps), _stream(f_a.device)))
        return f_a if nsteps % 2 == 0 else f_b

    def close(self):
        if getattr(self, "h", None):
            lib().lb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
