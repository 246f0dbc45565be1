"""torch.autograd.Function over the fused forward pass and its hand-written
adjoint (lasp_forward).

``SpectralObjective.apply(u, obs, ivar, basis, wave_grid, opts)`` returns, per
spectrum, J = chi2 / n_eff at the normalised parameters ``u`` [B, 5] with the
continuum at its weighted least-squares value (Eq. 6); its backward returns
dJ/du from the library's adjoint (envelope theorem: the continuum is held at
its optimum).  The only arithmetic here is autograd's chain rule, the
upstream gradient times the library's dJ/du.
"""

from __future__ import annotations

import torch

from . import lasp


class SpectralObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, obs, ivar, basis, wave_grid, opts: dict):
        res = lasp.forward(obs, ivar, wave_grid, basis, u.detach().contiguous(), want_grad=True,
                           **(opts or {}))
        ctx.save_for_backward(res["grad"])
        return res["J"]

    @staticmethod
    def backward(ctx, grad_J):
        (g,) = ctx.saved_tensors
        return grad_J.unsqueeze(1) * g, None, None, None, None, None


def objective(u, obs, ivar, basis, wave_grid, **opts):
    """J per spectrum, differentiable with respect to u."""
    return SpectralObjective.apply(u, obs, ivar, basis, wave_grid, opts)


def covariance(u, obs, ivar, basis, wave_grid, **opts):
    """Per-spectrum 5x5 covariance at u (physical units), from the forward-mode
    Jacobian and an FP64 Schur-complement inverse on the device."""
    return lasp.forward(obs, ivar, wave_grid, basis, u.detach().contiguous(), want_cov=True,
                        **opts)["cov"]
