"""Differentiable SPV trajectory observable for PyTorch.

`SPVTrajectory.apply(p0, x0, y0, theta0, L, params, T, ckpt_every)` runs T
steps of one periodic system from (x0, y0, theta0) with per-cell target shape
index p0 (P0_i = p0_i, A0 = 1) and returns Q = (1/T) sum_t mean_i P_i/sqrt(A_i)
as a 0-d tensor; its backward calls the library's checkpointed adjoint
(spv_traj_backward) and returns dQ/dp0.  The topology is held as recorded in
the forward pass (the derivative of the branch the trajectory took).
"""
from __future__ import annotations

import numpy as np
import torch

from . import spv


class SPVTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0, x0, y0, theta0, L, params, T, ckpt_every):
        p0n = p0.detach().to(torch.float64).cpu().numpy()
        s = spv.System(np.asarray(x0, dtype=np.float64), np.asarray(y0, dtype=np.float64), L, L, P0=p0n,
                       theta0=np.asarray(theta0, dtype=np.float64), params=params)
        Q = s.traj_forward(T, ckpt_every)
        ctx.sys = s
        ctx.p0_meta = (p0.dtype, p0.device)
        return torch.tensor(Q, dtype=p0.dtype, device=p0.device)

    @staticmethod
    def backward(ctx, gQ):
        s = ctx.sys
        g = s.traj_backward(float(gQ))
        s.close()
        dtype, device = ctx.p0_meta
        return torch.as_tensor(g, dtype=dtype, device=device), None, None, None, None, None, None, None


def trajectory_q(p0, x0, y0, theta0, L, params, T, ckpt_every):
    return SPVTrajectory.apply(p0, x0, y0, theta0, L, params, T, ckpt_every)
