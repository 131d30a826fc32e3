"""torch.autograd.Function over the library's cost and adjoint gradient."""

from __future__ import annotations

import torch

from . import api


class Chi2(torch.autograd.Function):
    """cost = Chi2.apply(params [n_vec, n_par] float64 CUDA tensor, ctx, data, theory, cost_kind).

    The forward pass runs the fused cost-and-gradient kernel once and keeps
    the gradient; backward scales it by the incoming gradient.  No second
    kernel launch and no finite differences."""

    @staticmethod
    def forward(fctx, params, ctx, data, theory, cost="chi2"):
        if not (params.is_cuda and params.dtype == torch.float64):
            raise TypeError("Chi2 needs a float64 tensor on the GPU")
        squeeze = params.dim() == 1
        p = params[None] if squeeze else params
        c, g = api.chi2_grad(ctx, data, theory, p, cost)
        fctx.save_for_backward(g)
        fctx.squeeze = squeeze
        return c[0] if squeeze else c

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        if fctx.squeeze:
            return grad_out * g[0], None, None, None, None
        return grad_out[:, None] * g, None, None, None, None
