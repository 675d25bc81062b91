"""torch.autograd.Function around gm_integrate_grad.

forward(theta) runs the adaptive cubature and the adjoint kernel in one call
and keeps dI/dtheta (the exact derivative of the quadrature over the frozen
region tree); backward returns grad_output * dI/dtheta.  theta is the params
vector a[0..d), u[0..d) as a float64 tensor (any device; the integration runs
on the current HIP device through the C ABI).
"""
from __future__ import annotations

import torch

from . import gm


class GMIntegral(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, family, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 22):
        p = theta.detach().to("cpu", torch.float64).numpy()
        est, err, grad, status = gm.integrate_grad(family, p, lo, hi, rel_tol, abs_tol,
                                                   max_regions)
        ctx.save_for_backward(torch.as_tensor(grad, dtype=theta.dtype, device=theta.device))
        ctx.status = status
        ctx.err = err
        return theta.new_tensor(est)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None, None, None


def integral(theta, family, lo, hi, rel_tol, abs_tol=1e-16, max_regions=1 << 22):
    """Differentiable integral of the family with parameters theta over [lo, hi]."""
    return GMIntegral.apply(theta, family, lo, hi, rel_tol, abs_tol, max_regions)
