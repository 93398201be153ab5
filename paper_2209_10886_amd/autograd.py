"""torch.autograd bridge: data misfit of Helmholtz solves as a differentiable function of m = 1/c^2.

Forward and adjoint solves both run in libhbj (hbj_gradient): A u_s = f_s, then
A mu_s = conj(P^T (P u_s - d_s)) with the same factors and preconditioner (A is
complex symmetric), and dL/dm accumulated on the GPU in FP64.  Only marshalling
happens here.
"""
from __future__ import annotations

import torch


class HelmholtzMisfit(torch.autograd.Function):
    """L(m) = 1/2 sum_s ||P u_s(m) - d_s||^2.

    forward(m, hctx, f, rec_idx, d, tol) -> scalar loss (float64 tensor on m's device);
    backward returns grad_out * dL/dm for m and None for the other inputs.
    ``hctx`` is a paper_2209_10886_amd.Context on the same grid; it is refactored for m.
    """

    @staticmethod
    def forward(ctx, m, hctx, f, rec_idx, d, tol=1e-10):
        hctx.set_slowness2(m.detach().to(torch.float64).contiguous())
        hctx.factor()
        loss, grad = hctx.gradient(f, rec_idx, d, tol=tol)
        ctx.save_for_backward(grad)
        return torch.tensor(loss, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad.to(grad_out.device), None, None, None, None, None


def misfit(m, hctx, f, rec_idx, d, tol=1e-10):
    return HelmholtzMisfit.apply(m, hctx, f, rec_idx, d, tol)
