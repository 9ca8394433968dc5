"""Differentiable pseudofermion action S = phi^dag (D^dag D)^{-1} phi, D = D_DW(m).

Forward: the adjoint solve Y = D^{-dag} phi, done with the multigrid solver as
Gamma5 D^{-1} Gamma5 phi (Gamma5-hermiticity, Sec. 2.1 of arXiv:2004.07732),
and S = |Y|^2.  Backward: X = D^{-1} Y and the outer-product force
    dS/dtheta_mu(x) = 2 Re sum_s [ i U Y_s(x)^dag (1-g_mu)/2 X_s(x+mu)
                                 - i U^* Y_s(x+mu)^dag (1+g_mu)/2 X_s(x) ]
from the force kernel.  Every solve, the Gamma5 maps, the norm and the force
run in the HIP library; this module only wires them into torch.autograd.
"""
from __future__ import annotations

import torch

from . import dwfmg


class DWFAction(torch.autograd.Function):
    """S(theta) for the hierarchy `mg` built (or updated) for U = exp(i theta)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, phi: torch.Tensor, mg: "dwfmg.MG", tol: float = 1e-12):
        U = dwfmg.dwf_links_from_theta(theta.detach().contiguous())
        mg.update_links(U)
        x, st = mg.solve(dwfmg.dwf_gamma5R(phi), tol)
        Y = dwfmg.dwf_gamma5R(x)
        S = dwfmg.dwf_norm2(Y.reshape(1, -1)).sum()
        ctx.mg, ctx.tol = mg, tol
        ctx.save_for_backward(U, Y)
        ctx.stats = st
        return S

    @staticmethod
    def backward(ctx, grad_out):
        U, Y = ctx.saved_tensors
        X, _ = ctx.mg.solve(Y, ctx.tol)
        F = dwfmg.dwf_force(U, X, Y)
        return grad_out * F, None, None, None


def action(theta: torch.Tensor, phi: torch.Tensor, mg: "dwfmg.MG", tol: float = 1e-12) -> torch.Tensor:
    return DWFAction.apply(theta, phi, mg, tol)
