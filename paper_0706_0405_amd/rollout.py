"""Gradients of a final-state loss with respect to the initial density.

The forward map is f^0 = f_eq(rho0, u0, p0/rho0) (lb_init), then N steps of
the scheme (lb_step), then the density readout rho_N = sum_i f_i^N. Its
reverse sweep uses the hand-written adjoint kernels: lb_step_adjoint for each
step (in reverse order) and lb_init_adjoint for the initial map. Only every
`seg`-th state is kept during the forward sweep (seg ~ sqrt(N)); the reverse
sweep recomputes one segment at a time from its checkpoint, so memory is
O(sqrt(N)) states for O(2N) forward steps. With keep_all=True every state is
kept instead (N + 1 arrays; a 2000-step FP32 rollout of a 960 x 240 grid takes
16.6 GB of device memory): the forward records them two steps per pass and the
reverse sweep needs no recomputation. The recorded states are bitwise those the
recomputation produces, so both ways give the same gradient bit for bit.
"""
from __future__ import annotations

import math

import torch

from . import api


class Rollout:
    """N-step rollout of one grid with fixed initial velocity and pressure fields."""

    def __init__(self, grid: api.Grid, ux0, uy0, p0, nsteps: int, prec="f32", seg=None, n0=0, keep_all=False):
        self.g, self.ux0, self.uy0, self.p0 = grid, ux0, uy0, p0
        self.n = int(nsteps)
        self.prec = prec
        self.n0 = int(n0)
        self.keep_all = bool(keep_all)
        self.seg = int(seg) if seg else max(1, int(round(math.sqrt(max(self.n, 1)))))

    # ------------------------------------------------------------ forward

    def _init(self, rho0):
        return api.init(self.g, rho0.detach().contiguous(), self.ux0, self.uy0, self.p0, prec=self.prec)

    def forward_density(self, rho0, checkpoints=None):
        """rho_N (ny, nx); if `checkpoints` is a list, the states f^(k seg) are appended to it."""
        g = self.g
        cur = self._init(rho0)
        if checkpoints is not None and self.keep_all and self.n > 0:
            # every state f^1 .. f^N recorded (two steps per pass); the list gets f^0 .. f^(N-1).
            # One allocation for all of them (a state's size is a multiple of 256 bytes, so
            # every view stays aligned): N separate allocations cost ~18 us each on the host.
            dt = api.DTYPE[api._prec(self.prec)]
            outs = list(torch.empty((self.n, 9, g.ny, g.pitch), dtype=dt, device=cur.device).unbind(0))
            api.run_record(g, cur, outs, n0=self.n0, prec=self.prec)
            checkpoints.extend([cur] + outs[:-1])
            return api.moments(g, outs[-1], prec=self.prec, flags=False)[0]
        nxt = api.empty(g, self.prec, cur.device)
        done = 0
        while done < self.n:
            if checkpoints is not None:
                checkpoints.append(cur.clone())
            k = min(self.seg, self.n - done)
            res = api.run(g, cur, nxt, k, n0=self.n0 + done, prec=self.prec)
            if res is nxt:
                cur, nxt = nxt, cur
            done += k
        rho = api.moments(g, cur, prec=self.prec, flags=False)[0]
        return rho

    # ------------------------------------------------------------ reverse

    def density_adjoint(self, rho0, g_rhoN, checkpoints):
        """dL/drho0 given dL/drho_N and the forward checkpoints."""
        g = self.g
        dev = g_rhoN.device
        # rho_N = sum_i f_i: the cotangent of every plane is dL/drho_N
        gbuf = api.empty(g, "f64", dev)
        gbuf.zero_()
        gbuf[:, :, :g.nx] = g_rhoN.to(torch.float64).unsqueeze(0)
        gtmp = api.empty(g, "f64", dev)
        gtmp.zero_()
        if self.keep_all and self.n > 0:   # checkpoints holds every state f^0 .. f^(N-1)
            res = api.adjoint_run(g, checkpoints, gbuf, gtmp, n0=self.n0, prec=self.prec)
            return api.init_adjoint(g, rho0.detach().to(torch.float64).contiguous(), self.ux0, self.uy0, self.p0, res)
        nseg = len(checkpoints)
        states = [None] * self.seg
        for s in reversed(range(nseg)):
            start = s * self.seg
            k = min(self.seg, self.n - start)
            # recompute the segment's states f^start .. f^(start+k-1), then sweep back over it
            for j in range(1, k):
                if states[j] is None:
                    states[j] = api.empty(g, self.prec, dev)
            seg_states = [checkpoints[s]] + states[1:k]
            if k > 1:
                api.run_record(g, checkpoints[s], seg_states[1:], n0=self.n0 + start, prec=self.prec)
            res = api.adjoint_run(g, seg_states, gbuf, gtmp, n0=self.n0 + start, prec=self.prec)
            if res is gtmp:
                gbuf, gtmp = gtmp, gbuf
        states.clear()
        return api.init_adjoint(g, rho0.detach().to(torch.float64).contiguous(), self.ux0, self.uy0, self.p0, gbuf)

    def loss_and_grad(self, rho0, target):
        """L = sum (rho_N - target)^2 and dL/drho0 through the autograd function."""
        r = rho0.detach().clone().requires_grad_(True)
        rhoN = RolloutFn.apply(r, self)
        loss = ((rhoN - target) ** 2).sum()
        loss.backward()
        return loss.detach(), r.grad


class RolloutFn(torch.autograd.Function):
    """rho_N = Rollout(rho0): forward through lb_init/lb_step, backward through
    lb_step_adjoint/lb_init_adjoint with sqrt(N) checkpoint recomputation."""

    @staticmethod
    def forward(ctx, rho0, roll: Rollout):
        cps = []
        rhoN = roll.forward_density(rho0, checkpoints=cps)
        ctx.roll = roll
        ctx.cps = cps
        ctx.save_for_backward(rho0)
        return rhoN

    @staticmethod
    def backward(ctx, g_rhoN):
        (rho0,) = ctx.saved_tensors
        grad = ctx.roll.density_adjoint(rho0, g_rhoN.contiguous(), ctx.cps)
        ctx.cps = None
        return grad, None
