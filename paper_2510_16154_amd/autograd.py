"""Differentiable agent dynamics: a torch.autograd.Function over the HIP library.

Forward runs ``abc_forward_dynamics`` (K explicit Euler steps of the
windowed agent dynamics) and keeps either the whole trajectory or, with
``params.ckpt_every = k``, one state every k steps.  Backward runs
``abc_adjoint_dynamics``: the discrete adjoint (transposed Jacobians of
Sec. 3.1), recomputing each checkpointed segment once, and returns
dl/dc0 and dl/deps.  Marshalling only; all arithmetic is in the library.
"""
from __future__ import annotations

import torch

from .binding import Params, abc_adjoint_dynamics, abc_forward_dynamics


class AgentDynamics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c0: torch.Tensor, eps: torch.Tensor, params: Params):
        c0c = c0.detach().contiguous()
        epsc = eps.detach().contiguous()
        traj = abc_forward_dynamics(c0c, epsc, params)
        ctx.save_for_backward(traj, epsc)
        ctx.params = params
        return traj[-1].clone()

    @staticmethod
    def backward(ctx, gK: torch.Tensor):
        traj, eps = ctx.saved_tensors
        g0, geps = abc_adjoint_dynamics(traj, eps, ctx.params, gK.contiguous())
        return g0, geps, None


def agent_dynamics(c0: torch.Tensor, eps: torch.Tensor, params: Params) -> torch.Tensor:
    """c(T) of the agent dynamics from c0 (H x W x C) under controls eps (K x 2), differentiable in both."""
    return AgentDynamics.apply(c0, eps, params)
