"""Gradient of the mean hot-wall Nusselt number after N pseudo-time steps
with respect to the hot-wall temperatures Theta (one per wall row) and Ra,
by the library's discrete adjoint (cavity_nusselt_adjoint,
cavity_adjoint_step) with step checkpointing.

The forward run keeps the state every `every` steps (the checkpoints).  The
reverse sweep walks the segments last to first: it recomputes the states of
one segment from its checkpoint with cavity_step, then runs the reverse steps
of that segment.  The recomputation of the next segment runs on a second
stream while the reverse steps of the current one run, into the other of two
segment buffers.  Memory: N/every checkpoints plus two segments of states;
work: two forward runs plus N reverse steps.  Every step, forward or
reverse, runs in the library's kernels; this module only orders the calls
and holds torch buffers.
"""
import dataclasses
from typing import List, Optional, Tuple

from . import (CAV_F64, Grid, Params, cavity_adjoint_step, cavity_adjoint_workspace_bytes,
               cavity_nusselt, cavity_nusselt_adjoint, cavity_state_elems, cavity_step, cavity_step_from,
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
    gradient (dJ/dtheta, dJ/dRa, dJ/dq0).

    All buffers (checkpoints, one segment of states, cotangents, wall field)
    are allocated once per device and reused, so a backward pass allocates
    nothing.  With graph=True the backward pass is captured into one HIP
    graph the first time it runs at a given Ra and replayed afterwards (its
    launches hold Ra's coefficients and the buffers' addresses, which do not
    change between calls)."""

    def __init__(self, grid: Grid, params: Params, nsteps: int, every: int = 20, graph: bool = False):
        if grid.dtype != CAV_F64:
            raise ValueError("the adjoint is available for FP64 grids only")
        self.grid, self.nsteps, self.every = grid, int(nsteps), int(every)
        self.base = params
        self.segs = segments(self.nsteps, self.every)
        self.graph = bool(graph)
        self.prm: Optional[Params] = None
        self._b = None            # persistent buffers
        self._g = None            # captured backward graph
        self._g_ra = None         # the Ra it was captured at

    def _buffers(self, device):
        import torch
        if self._b is not None and self._b["dev"] == device:
            return self._b
        g = self.grid
        n = cavity_state_elems(g)
        f64 = dict(dtype=torch.float64, device=device)
        self._b = dict(
            dev=device,
            ckpt=torch.zeros((max(len(self.segs), 1), n), **f64),
            states=torch.zeros((2, max(self.every - 1, 1), n), **f64),
            q=torch.zeros(n, **f64), tmp=torch.zeros(n, **f64),
            ws=torch.zeros(cavity_workspace_bytes(g) // 8, **f64),
            lam=(torch.zeros(n, **f64), torch.zeros(n, **f64)),
            dth=torch.zeros(g.nj * g.nk, **f64), dra=torch.zeros(1, **f64),
            aws=torch.zeros(cavity_adjoint_workspace_bytes(g) // 8, **f64),
            theta=torch.zeros(g.nj * g.nk, **f64),
            side=torch.cuda.Stream(device=device))
        self._g = None
        return self._b

    def forward(self, theta, Ra: float, q0) -> float:
        """Runs the N steps from q0 (flat state tensor, library layout),
        keeping the checkpoints; returns J."""
        B = self._buffers(q0.device)
        B["theta"].copy_(theta.detach().reshape(-1))
        self.prm = dataclasses.replace(self.base, Ra=float(Ra), t_hot_field=B["theta"])
        q = B["q"]
        q.copy_(q0.detach())
        for s, (_, length) in enumerate(self.segs):
            B["ckpt"][s].copy_(q)
            cavity_step(self.grid, self.prm, None, q, B["tmp"], B["ws"], None, length)
        self.J = cavity_nusselt(self.grid, self.prm, q, B["ws"])
        return self.J

    def _recompute(self, s: int, b: int):
        """The states of segment s, recomputed from its checkpoint into
        segment buffer b on the current stream (its first state is the
        checkpoint itself)."""
        B, g, prm = self._b, self.grid, self.prm
        states = [B["ckpt"][s]]
        for m in range(1, self.segs[s][1]):
            st = B["states"][b][m - 1]
            cavity_step_from(g, prm, states[-1], st)
            states.append(st)
        return states

    def _reverse(self):
        """Every launch of the backward pass, issued from the current stream:
        seed the cotangent of J, then per segment (last to first) run its
        reverse steps over its recomputed states.  The states of the next
        segment are recomputed on a second stream meanwhile, into the other
        segment buffer (once the reverse steps that read that buffer before
        are done); the current stream waits for them before using them and
        joins the second stream at the end.  The cotangent alternates between
        two buffers (a reverse step reads its input at every cell's
        neighbours, so it cannot write in place); after N steps it is in
        buffer N mod 2."""
        import torch
        B, g, prm = self._b, self.grid, self.prm
        lam, dth, dra = B["lam"], B["dth"], B["dra"]
        main, side = torch.cuda.current_stream(), B["side"]
        dth.zero_()
        dra.zero_()
        cur = 0
        cavity_nusselt_adjoint(g, prm, lam[cur], dth)
        order = list(reversed(range(len(self.segs))))
        if not order:
            return
        states = self._recompute(order[0], 0)
        side.wait_stream(main)
        free = [None, None]              # main has finished reading buffer b
        done = [None, None]              # side has finished writing buffer b
        nxt = None
        for idx, s in enumerate(order):
            b = idx % 2
            if idx + 1 < len(order):
                with torch.cuda.stream(side):
                    if free[1 - b] is not None:
                        side.wait_event(free[1 - b])
                    nxt = self._recompute(order[idx + 1], 1 - b)
                    done[1 - b] = torch.cuda.Event()
                    done[1 - b].record(side)
            if idx > 0:
                main.wait_event(done[b])
            for st in reversed(states):
                cavity_adjoint_step(g, prm, st, lam[cur], lam[1 - cur], B["aws"], dth, dra)
                cur = 1 - cur
            free[b] = torch.cuda.Event()
            free[b].record(main)
            states = nxt
        main.wait_stream(side)

    def backward(self):
        """(dJ/dtheta (nj*nk), dJ/dRa (1), dJ/dq0 (flat state, zero ghosts))."""
        import torch
        if self.prm is None:
            raise RuntimeError("forward() must run first")
        B = self._b
        if not self.graph:
            self._reverse()
        elif self._g is not None and self._g_ra == self.prm.Ra:
            self._g.replay()
        else:
            # first pass at this Ra: run it (the results), then capture it
            # (capture records the launches without running them)
            self._g = None
            self._reverse()
            gr = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gr):
                self._reverse()
            self._g, self._g_ra = gr, self.prm.Ra
        g = self.grid
        lam = B["lam"][self.nsteps % 2]
        dq0 = torch.zeros_like(lam)
        G = g.ng
        inner = (slice(None), slice(G, G + g.nk), slice(G, G + g.nj), slice(G, G + g.ni))
        state_view(g, dq0)[inner] = state_view(g, lam)[inner]
        return B["dth"].clone(), B["dra"].clone(), dq0


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
