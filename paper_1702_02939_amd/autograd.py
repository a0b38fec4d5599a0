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


def _f64(a):
    # tensors (host or device) go to the library as they are, anything else
    # as a float64 numpy array
    if isinstance(a, torch.Tensor):
        return a.detach().to(torch.float64).contiguous()
    return np.asarray(a, dtype=np.float64)


class SPVTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p0, x0, y0, theta0, L, params, T, ckpt_every):
        # p0 stays where it is (the library reads host or device memory)
        s = spv.System(_f64(x0), _f64(y0), L, L, P0=_f64(p0), theta0=_f64(theta0), params=params)
        Q = s.traj_forward(T, ckpt_every)
        ctx.sys = s
        ctx.p0_meta = (p0.dtype, p0.device)
        return torch.tensor(Q, dtype=p0.dtype, device=p0.device)

    @staticmethod
    def backward(ctx, gQ):
        s = ctx.sys
        dtype, device = ctx.p0_meta
        g = torch.empty(s.N, dtype=torch.float64, device=device)  # written by the library in place
        s.traj_backward(float(gQ), g)
        s.close()
        return g.to(dtype), None, None, None, None, None, None, None


def trajectory_q(p0, x0, y0, theta0, L, params, T, ckpt_every):
    return SPVTrajectory.apply(p0, x0, y0, theta0, L, params, T, ckpt_every)
