"""Pade Jastrow parameters theta = (b_ee, b_en) behind torch.autograd.

PadeJastrow.apply(theta, engine, pos) returns, for the walker configurations
pos of an LRDMC context, the Jastrow exponent J and the local energy E_L
evaluated at theta; the backward pass contracts the output gradients with
dJ/dtheta and dE_L/dtheta from the HIP gradient kernel (lrdmc_jastrow_grad).
The forward pass sets the context's parameters to theta (lrdmc_set_jastrow).

vmc_variance_step is one step of variance minimisation of E_L over fixed
configurations sampled at theta0, with the correlated-sampling weights
|Psi_theta / Psi_theta0|^2 = exp(2 (J_theta - J_theta0)): the objective uses
both outputs, so gradients flow through both kernel derivatives.
"""
from __future__ import annotations

import torch

from .lrdmc import LRDMC, lrdmc_jastrow_grad, lrdmc_set_jastrow


class PadeJastrow(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, engine: LRDMC, pos: torch.Tensor):
        b = theta.detach().to("cpu", torch.float64)
        pos = engine.positions(pos)
        lrdmc_set_jastrow(engine.ctx, float(b[0]), float(b[1]))
        out = torch.empty(engine.W, 6, dtype=torch.float64, device=engine.device)
        lrdmc_jastrow_grad(engine.ctx, pos, out)
        ctx.save_for_backward(out[:, 2:6].clone())
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        return out[:, 1].clone(), out[:, 0].clone()

    @staticmethod
    def backward(ctx, g_j, g_e):
        (d,) = ctx.saved_tensors
        grad = torch.zeros(2, dtype=torch.float64, device=d.device)
        if g_j is not None:
            grad = grad + (g_j[:, None] * d[:, 0:2]).sum(0)
        if g_e is not None:
            grad = grad + (g_e[:, None] * d[:, 2:4]).sum(0)
        return grad.to(ctx.theta_device, ctx.theta_dtype), None, None


def jastrow_and_local_energy(theta: torch.Tensor, engine: LRDMC, pos: torch.Tensor):
    """(J[W], E_L[W]) at theta, differentiable in theta."""
    return PadeJastrow.apply(theta, engine, pos)


def weighted_variance(theta: torch.Tensor, engine: LRDMC, pos: torch.Tensor, j0: torch.Tensor):
    """Variance of E_L under |Psi_theta|^2 estimated on configurations sampled
    from |Psi_theta0|^2 (j0 = J at theta0), and the weighted mean energy."""
    j, e = jastrow_and_local_energy(theta, engine, pos)
    lw = 2.0 * (j - j0)
    w = torch.exp(lw - lw.max())
    w = w / w.sum()
    e_mean = (w * e).sum()
    return (w * (e - e_mean) ** 2).sum(), e_mean
