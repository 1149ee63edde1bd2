"""torch.autograd bindings of the HIP step and its hand-written adjoint.

StepFn.apply(prims, gamma, solver, dt) advances padded prims by one SSPRK2
step; its backward calls grmhd_step_vjp, which recomputes the step from the
saved input prims (one checkpoint per step) and returns the adjoint of the
prims and of the adiabatic index.  run(...) chains steps.
"""

import torch

from . import grmhd as gr


class StepFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prims, gamma, solver, dt):
        g = float(gamma)
        if abs(g - solver.params.gamma_ad) > 0.0:
            raise gr.GrmhdError("gamma must equal the solver's gamma_ad")
        solver.load(prims.detach())
        solver.step(dt)
        out = solver.prims()
        ctx.save_for_backward(prims.detach())
        ctx.solver, ctx.dt = solver, dt
        return out

    @staticmethod
    def backward(ctx, gout):
        (prims,) = ctx.saved_tensors
        gin, ggam = ctx.solver.step_vjp(prims, ctx.dt, gout.contiguous())
        return gin, torch.tensor(ggam, dtype=torch.float64, device=gin.device), None, None


def run(prims, gamma, solver, dt, nsteps):
    """nsteps chained steps with per-step checkpoints."""
    p = prims
    for _ in range(nsteps):
        p = StepFn.apply(p, gamma, solver, dt)
    return p
