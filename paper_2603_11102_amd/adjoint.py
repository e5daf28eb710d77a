"""torch.autograd.Function over a window of S2O4 steps: mean rotor power and thrust as functions of
the per-actuator-point force scalings, with the hand-written adjoint of libgks.so as the backward.

Forward: an FP64 context on the GPU steps the window from the case's initial field, storing one
checkpoint per step. Backward: gks_adjoint recomputes every step from its checkpoint and runs the
reverse sweep (WENO nonlinear weights frozen at their forward values, or differentiated as well with
``exact=True``).
"""
from __future__ import annotations

import torch

from .solver import GksSolver


class RotorWindow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, scales: torch.Tensor, cfg, nsteps: int, exact: bool = False):
        s = GksSolver(cfg, precision="fp64", device=scales.device)
        sc = scales.detach().to(torch.float64).contiguous()
        s.set_rotor(cfg.rotor, scale=sc)
        s.set_checkpoints(nsteps)
        s.step(nsteps)
        f = s.forces()
        n = f["window_steps"]
        out = torch.tensor([f["window_power"] / n, f["window_thrust"] / n], dtype=torch.float64,
                           device=scales.device)
        ctx.solver = s
        ctx.nsteps = nsteps
        ctx.keep = sc
        ctx.exact = exact
        return out

    @staticmethod
    def backward(ctx, grad_out):
        w = grad_out.detach().to(torch.float64).cpu().tolist()
        g, _ = ctx.solver.adjoint(ctx.nsteps, w, exact=ctx.exact)
        ctx.solver.close()
        return g.to(grad_out.device), None, None, None


def rotor_window(scales: torch.Tensor, cfg, nsteps: int, exact: bool = False) -> torch.Tensor:
    """[mean P, mean T] over nsteps steps; differentiable with respect to ``scales`` (``exact``: the
    WENO weights are differentiated too)."""
    return RotorWindow.apply(scales, cfg, nsteps, exact)
