"""torch.autograd face of the hand-written adjoint.

``ssprk3(solver, U0, dts, every)`` runs len(dts) SSP-RK3 steps with the
given (frozen) time steps and returns the final state; its backward is the
library's reverse sweep (idp_adjoint_checkpoints): each segment of
``every`` steps is recomputed from a checkpoint and stepped backwards, so
the graph viscosity, the bounds and the limiter coefficients are
recomputed in the backward, never stored for the whole run.

The solver keeps the checkpoints of its latest forward_checkpoints run only.
Each forward records which run it was (the solver's checkpoint generation)
and its initial state; a backward whose run is no longer the latest (another
ssprk3 or forward_checkpoints on the same solver came between) first redoes
its own forward from that state, so it never differentiates another run.
"""
from __future__ import annotations

import numpy as np
import torch


class _SSPRK3Steps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dts, every):
        start = U0.detach().clone().contiguous()
        U = start.clone()
        solver.forward_checkpoints(U, dts, every)
        ctx.solver, ctx.dts, ctx.every = solver, dts, every
        ctx.start, ctx.generation = start, solver.checkpoint_generation
        return U

    @staticmethod
    def backward(ctx, Ubar):
        s = ctx.solver
        if s.checkpoint_generation != ctx.generation:
            # another run replaced this one's checkpoints: recompute them
            U = ctx.start.clone()
            s.forward_checkpoints(U, ctx.dts, ctx.every)
            ctx.generation = s.checkpoint_generation
        g = s.adjoint_checkpoints(ctx.dts, ctx.every, Ubar.contiguous())
        return g, None, None, None


def ssprk3(solver, U0, dts, every: int = 20):
    """Final state after the steps dts (differentiable w.r.t. U0)."""
    d = np.ascontiguousarray(dts, dtype=np.float64)
    return _SSPRK3Steps.apply(U0, solver, d, int(every))
