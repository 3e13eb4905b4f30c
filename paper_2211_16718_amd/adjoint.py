"""Gradient of the final kinetic energy with respect to the initial velocity.

``FinalKineticEnergy.apply(v0, rho0, p0, plan, dt, nsteps, ckpt_every[, scheme])``
returns J = <|m|^2 / (2 rho)> after ``nsteps`` steps of ``scheme`` ("rk4", the
default, or "tvdrk3") from the state built from the primitives (rho0, v0, p0); its
backward gives dJ/dv0 at fixed rho0 and p0.  The
forward call runs the library's checkpointed adjoint (a forward pass storing
checkpoints every ``ckpt_every`` steps, then the reverse sweep with segment
recomputation), so the backward only applies the transpose of the initial-state
map on the device.
"""
from __future__ import annotations

import torch


class FinalKineticEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v0, rho0, p0, plan, dt, nsteps, ckpt_every, scheme="rk4"):
        v0c = v0.detach().to(device=plan.device, dtype=torch.float64).contiguous()
        rho = rho0.detach().to(device=plan.device, dtype=torch.float64).contiguous()
        p = p0.detach().to(device=plan.device, dtype=torch.float64).contiguous()
        u0 = plan.init_state(rho, v0c, p)
        run = {"rk4": plan.adjoint_rk4, "tvdrk3": plan.adjoint_tvdrk3}[scheme]
        J, u0bar = run(u0, dt, nsteps, ckpt_every)
        ctx.plan = plan
        ctx.save_for_backward(rho, v0c, u0bar)
        return J[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        rho, v0, u0bar = ctx.saved_tensors
        vbar = ctx.plan.ic_vjp(rho, v0, u0bar)
        return gJ * vbar, None, None, None, None, None, None, None
