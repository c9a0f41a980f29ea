"""torch.autograd binding of the applied dual operator.

q = F(theta) lambda with F = sum_i D_i^T B~_i K_reg,i(theta)^{-1} B~_i^T D_i.
The forward calls fetiF_apply; the backward calls fetiF_apply_backward,
which returns dlambda = F g (F is symmetric) and
dtheta_e = -u_g|_e^T (dK_reg/dtheta_e) u_lambda|_e with u_x = K_reg^{-1} B~^T D x.

theta enters the operator through the host factorisation: the context must
have been factored and assembled for the theta passed here (fetiF_create
with element data, fetiF_factor_upload, fetiF_assemble); theta is an input
of the Function only so that autograd routes its gradient.
"""
from __future__ import annotations

import torch


class FetiApply(torch.autograd.Function):
    @staticmethod
    def forward(fctx, lam, theta, feti):
        lam = lam.contiguous()
        q = torch.empty(lam.shape, dtype=lam.dtype, device=lam.device)
        feti.apply(lam, q)
        fctx.feti = feti
        fctx.theta_shape = theta.shape
        fctx.save_for_backward(lam)
        return q

    @staticmethod
    def backward(fctx, g):
        (lam,) = fctx.saved_tensors
        feti = fctx.feti
        g = g.contiguous()
        dlam = torch.empty(lam.shape, dtype=lam.dtype, device=lam.device)
        dth = None
        if fctx.needs_input_grad[1]:
            dth = torch.empty(fctx.theta_shape, dtype=lam.dtype, device=lam.device)
        feti.apply_backward(g, lam, dlam, dth)
        return (dlam if fctx.needs_input_grad[0] else None), dth, None


def feti_apply(lam, theta, feti):
    """q = F(theta) lambda, differentiable in lambda and theta."""
    return FetiApply.apply(lam, theta, feti)
