"""torch.autograd.Function around the library's discrete adjoint.

J(a) = integral of u_h(T)^2 after n_steps implicit-Euler steps of the
two-scale system from a fixed initial state, as a function of the
per-instance deformation amplitudes a.  forward() runs tsm_gradient (forward
with checkpoints plus the adjoint sweep) and keeps dJ/da; backward() scales
it by the incoming gradient.  All arithmetic runs in libtsm.
"""
from __future__ import annotations

import torch


class TwoScaleObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, batch, u0, v0, n_steps):
        batch.set_deformation(a.detach())
        batch.set_state(u0, v0)
        J, g = batch.gradient(int(n_steps))
        ctx.save_for_backward(g)
        return torch.tensor(J, dtype=torch.float64, device=a.device)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return gJ * g, None, None, None, None


def objective(a, batch, u0, v0, n_steps):
    """J(a) with autograd support (see TwoScaleObjective)."""
    return TwoScaleObjective.apply(a, batch, u0, v0, n_steps)
