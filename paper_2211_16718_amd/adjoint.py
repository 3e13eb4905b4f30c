"""Gradient of the final kinetic energy with respect to the initial velocity.

``FinalKineticEnergy.apply(v0, rho0, p0, plan, dt, nsteps, ckpt_every[, scheme])``
returns J = <|m|^2 / (2 rho)> after ``nsteps`` steps of ``scheme`` ("rk4", the
default, or "tvdrk3") from the state built from the primitives (rho0, v0, p0); its
backward gives dJ/dv0 at fixed rho0 and p0.  The forward call runs the library's
forward pass only (the steps, with a checkpoint every ``ckpt_every`` steps, kept in
a workspace of its own); the backward call runs the reverse sweep from that workspace
(segments recomputed from their checkpoints) and applies the transpose of the
initial-state map, all on the device.
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
        ws = plan.adjoint_workspace(nsteps, ckpt_every)
        J = plan.adjoint_forward(u0, dt, nsteps, ckpt_every, ws, scheme)
        ctx.plan = plan
        ctx.args = (dt, nsteps, ckpt_every, scheme)
        ctx.ws = ws
        ctx.save_for_backward(rho, v0c)
        return J[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        rho, v0 = ctx.saved_tensors
        dt, nsteps, ckpt_every, scheme = ctx.args
        u0bar = ctx.plan.adjoint_reverse(dt, nsteps, ckpt_every, ctx.ws, scheme)
        ctx.ws = None  # release the checkpoints
        vbar = ctx.plan.ic_vjp(rho, v0, u0bar)
        return gJ * vbar, None, None, None, None, None, None, None
