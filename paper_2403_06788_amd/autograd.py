"""torch.autograd.Function over the library's adjoint kernels.

J = DSGRFTObjective.apply(plan, echo, theta) gives J_b = |Y(theta_b)|^2 for
candidates theta [B, 3] = (r0, v, a); backward returns dJ/dtheta (FP64) and
dJ/decho (complex64, PyTorch's convention for complex inputs).  Both
directions run in the HIP kernels of libdsgrft.
"""
from __future__ import annotations

import torch


class DSGRFTObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, echo, theta):
        J, saved = plan.adjoint_forward(echo, theta)
        ctx.plan = plan
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        ctx.save_for_backward(echo, theta.detach().to(torch.float64), saved)
        return J

    @staticmethod
    def backward(ctx, gJ):
        echo, theta, saved = ctx.saved_tensors
        need_echo, need_theta = ctx.needs_input_grad[1], ctx.needs_input_grad[2]
        gt, ge = ctx.plan.adjoint_backward(echo, theta, saved, gJ.contiguous(),
                                           want_theta=need_theta, want_echo=need_echo)
        if gt is not None:
            # the gradient goes back on theta's own device and in its dtype
            gt = gt.to(device=ctx.theta_device, dtype=ctx.theta_dtype)
        return None, ge, gt


def objective(plan, echo, theta):
    return DSGRFTObjective.apply(plan, echo, theta)
