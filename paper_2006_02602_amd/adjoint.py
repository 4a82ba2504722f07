"""Gradient of the mean hot-wall Nusselt number after N pseudo-time steps
with respect to the hot-wall temperatures Theta (one per wall row) and Ra,
by the library's discrete adjoint (cavity_nusselt_adjoint,
cavity_adjoint_step) with step checkpointing.

The forward run keeps the state every `every` steps (the checkpoints).  The
reverse sweep walks the segments last to first: it recomputes the states of
one segment from its checkpoint with cavity_step, then runs the reverse steps
of that segment.  Memory: N/every checkpoints plus one segment of states;
work: two forward runs plus N reverse steps.  Every step, forward or
reverse, runs in the library's kernels; this module only orders the calls
and holds torch buffers.
"""
import dataclasses
from typing import List, Optional, Tuple

from . import (CAV_F64, Grid, Params, cavity_adjoint_step, cavity_adjoint_workspace_bytes,
               cavity_nusselt, cavity_nusselt_adjoint, cavity_state_elems, cavity_step,
               cavity_workspace_bytes, state_view)


def segments(nsteps: int, every: int) -> List[Tuple[int, int]]:
    """Checkpoint segments (first step, length) in forward order; the last
    one may be shorter."""
    if nsteps < 0 or every < 1:
        raise ValueError("nsteps must be >= 0 and every >= 1")
    return [(s, min(every, nsteps - s)) for s in range(0, nsteps, every)]


class NusseltAdjoint:
    """J = Nu(q^N) of the cavity started from q0 with hot-wall temperatures
    theta and Rayleigh number Ra; forward() returns J, backward() the
    gradient (dJ/dtheta, dJ/dRa, dJ/dq0)."""

    def __init__(self, grid: Grid, params: Params, nsteps: int, every: int = 20):
        if grid.dtype != CAV_F64:
            raise ValueError("the adjoint is available for FP64 grids only")
        self.grid, self.nsteps, self.every = grid, int(nsteps), int(every)
        self.base = params
        self.segs = segments(self.nsteps, self.every)
        self.ckpt = []
        self.prm: Optional[Params] = None

    def _buffers(self, device):
        import torch
        n = cavity_state_elems(self.grid)
        tmp = torch.empty(n, dtype=torch.float64, device=device)
        ws = torch.zeros(cavity_workspace_bytes(self.grid) // 8, dtype=torch.float64, device=device)
        return tmp, ws

    def forward(self, theta, Ra: float, q0) -> float:
        """Runs the N steps from q0 (flat state tensor, library layout),
        keeping the checkpoints; returns J."""
        self.theta = theta.detach().contiguous()
        self.prm = dataclasses.replace(self.base, Ra=float(Ra), t_hot_field=self.theta)
        tmp, ws = self._buffers(q0.device)
        q = q0.detach().clone()
        self.ckpt = []
        for _, length in self.segs:
            self.ckpt.append(q.clone())
            cavity_step(self.grid, self.prm, None, q, tmp, ws, None, length)
        self.J = cavity_nusselt(self.grid, self.prm, q, ws)
        return self.J

    def backward(self):
        """(dJ/dtheta (nj*nk), dJ/dRa (1), dJ/dq0 (flat state, zero ghosts))."""
        import torch
        if self.prm is None:
            raise RuntimeError("forward() must run first")
        g, prm = self.grid, self.prm
        dev = self.ckpt[0].device if self.ckpt else self.theta.device
        n = cavity_state_elems(g)
        lam = torch.zeros(n, dtype=torch.float64, device=dev)
        dth = torch.zeros(g.nj * g.nk, dtype=torch.float64, device=dev)
        dra = torch.zeros(1, dtype=torch.float64, device=dev)
        aws = torch.empty(cavity_adjoint_workspace_bytes(g) // 8, dtype=torch.float64, device=dev)
        tmp, ws = self._buffers(dev)
        cavity_nusselt_adjoint(g, prm, lam, dth)
        for (_, length), ck in zip(reversed(self.segs), reversed(self.ckpt)):
            states = [ck]
            for _ in range(length - 1):
                s = states[-1].clone()
                cavity_step(g, prm, None, s, tmp, ws, None, 1)
                states.append(s)
            for s in reversed(states):
                cavity_adjoint_step(g, prm, s, lam, lam, aws, dth, dra)
        dq0 = torch.zeros_like(lam)
        G = g.ng
        inner = (slice(None), slice(G, G + g.nk), slice(G, G + g.nj), slice(G, G + g.ni))
        state_view(g, dq0)[inner] = state_view(g, lam)[inner]
        return dth, dra, dq0


def _function():
    import torch

    class NusseltFunction(torch.autograd.Function):
        """J = Nu(q^N) as a differentiable function of (theta, Ra, q0)."""

        @staticmethod
        def forward(ctx, theta, ra, q0, grid, params, nsteps, every):
            adj = NusseltAdjoint(grid, params, nsteps, every)
            J = adj.forward(theta, float(ra), q0)
            ctx.adj = adj
            ctx.ra_dev = ra.device
            return torch.tensor(J, dtype=torch.float64, device=theta.device)

        @staticmethod
        def backward(ctx, gJ):
            dth, dra, dq0 = ctx.adj.backward()
            ctx.adj = None
            gj = gJ.to(dth.device)
            return gj * dth, (gj * dra[0]).to(ctx.ra_dev), gj * dq0, None, None, None, None

    return NusseltFunction


_NUSSELT_FN = None


def nusselt(theta, ra, q0, grid: Grid, params: Params, nsteps: int, every: int = 20):
    """Differentiable J = mean hot-wall Nusselt number after `nsteps` steps
    from q0 (torch.autograd): theta (nj*nk float64 GPU tensor), ra (0-d
    float64 tensor), q0 (flat float64 GPU state in the library layout)."""
    global _NUSSELT_FN
    if _NUSSELT_FN is None:
        _NUSSELT_FN = _function()
    return _NUSSELT_FN.apply(theta, ra, q0, grid, params, nsteps, every)
