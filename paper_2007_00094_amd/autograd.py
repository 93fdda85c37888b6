"""torch.autograd face of the hand-written adjoint.

``ssprk3(solver, U0, dts, every)`` runs len(dts) SSP-RK3 steps with the
given (frozen) time steps and returns the final state; its backward is the
library's reverse sweep (idp_adjoint_checkpoints): each segment of
``every`` steps is recomputed from a checkpoint and stepped backwards, so
the graph viscosity, the bounds and the limiter coefficients are
recomputed in the backward, never stored for the whole run.
"""
from __future__ import annotations

import numpy as np
import torch


class _SSPRK3Steps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dts, every):
        U = U0.detach().clone().contiguous()
        solver.forward_checkpoints(U, dts, every)
        ctx.solver, ctx.dts, ctx.every = solver, dts, every
        return U

    @staticmethod
    def backward(ctx, Ubar):
        g = ctx.solver.adjoint_checkpoints(ctx.dts, ctx.every, Ubar.contiguous())
        return g, None, None, None


def ssprk3(solver, U0, dts, every: int = 20):
    """Final state after the steps dts (differentiable w.r.t. U0)."""
    d = np.ascontiguousarray(dts, dtype=np.float64)
    return _SSPRK3Steps.apply(U0, solver, d, int(every))
