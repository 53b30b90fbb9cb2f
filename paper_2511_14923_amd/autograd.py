"""torch.autograd.Function over libgbs, and the differentiable covariance model.

GBSCumulants.apply(sigma, max_order, flags) -> (corr, cum) runs gbs_cumulants;
its backward runs the library's adjoint kernels (gbs_cumulant_grad) and returns
dL/dsigma, which torch then chains through whatever produced sigma.

lossy_squeezed_covariance(W, r, eta) builds the output covariance (xxpp,
hbar = 1) of M x-squeezed vacua with input-side transmissions eta sent through
the interferometer whose symplectic matrix is W (App. F, Eqs.
jiuzhang_input_cov, symplectic_inter, ground_truth_cov with T = U diag(sqrt(eta))):
    sigma = W diag(eta e^{-2r}/2 + (1-eta)/2, eta e^{2r}/2 + (1-eta)/2) W^T,
differentiable in (r, eta), so a cumulant-matching loss can fit per-mode
transmissions and squeezings.
"""
from __future__ import annotations

import torch

from ._binding import (GBS_MIXED, GBS_PARITY, gbs_cumulant_grad, gbs_cumulants,
                       gbs_total_outputs)


class GBSCumulants(torch.autograd.Function):
    """(corr, cum) = GBSCumulants.apply(sigma, max_order, flags)."""

    @staticmethod
    def forward(ctx, sigma, max_order: int, flags: int = 0):
        sigma = sigma.contiguous()
        M = sigma.shape[0] // 2
        corr, cum = gbs_cumulants(M, sigma, max_order, flags)
        ctx.save_for_backward(sigma)
        ctx.max_order = max_order
        ctx.flags = flags
        return corr, cum

    @staticmethod
    def backward(ctx, g_corr, g_cum):
        (sigma,) = ctx.saved_tensors
        if ctx.flags & GBS_MIXED:
            raise RuntimeError("the adjoint is FP64 only: run the forward without GBS_MIXED")
        M = sigma.shape[0] // 2
        n = gbs_total_outputs(M, ctx.max_order)
        gc = g_corr.contiguous() if g_corr is not None else None
        gk = g_cum.contiguous() if g_cum is not None else None
        if gc is not None and gc.numel() != n or gk is not None and gk.numel() != n:
            raise ValueError("upstream gradient has the wrong size")
        g_sigma = gbs_cumulant_grad(M, sigma, ctx.max_order, ctx.flags & GBS_PARITY,
                                    grad_corr=gc, grad_cum=gk)
        return g_sigma, None, None


def cumulants(sigma: torch.Tensor, max_order: int, flags: int = 0):
    """Differentiable (corr, cum) of a device FP64 covariance."""
    return GBSCumulants.apply(sigma, max_order, flags)


def interferometer_symplectic(U: torch.Tensor) -> torch.Tensor:
    """[[Re U, -Im U], [Im U, Re U]] (Eq. symplectic_inter)."""
    re, im = U.real, U.imag
    return torch.cat([torch.cat([re, -im], 1), torch.cat([im, re], 1)], 0).contiguous()


def lossy_squeezed_covariance(W: torch.Tensor, r: torch.Tensor, eta: torch.Tensor) -> torch.Tensor:
    """sigma(r, eta) for a fixed interferometer symplectic W (2M x 2M, FP64)."""
    sx = 0.5 * eta * torch.exp(-2.0 * r) + 0.5 * (1.0 - eta)
    sp = 0.5 * eta * torch.exp(2.0 * r) + 0.5 * (1.0 - eta)
    d = torch.cat([sx, sp])
    sigma = (W * d.unsqueeze(0)) @ W.T
    return 0.5 * (sigma + sigma.T)


def cumulant_matching_loss(W: torch.Tensor, r: torch.Tensor, eta: torch.Tensor,
                           target_cum: torch.Tensor, max_order: int) -> torch.Tensor:
    """sum over all |S| <= max_order of (kappa~(S; r, eta) - target(S))^2."""
    sigma = lossy_squeezed_covariance(W, r, eta)
    _, cum = cumulants(sigma, max_order)
    return ((cum - target_cum) ** 2).sum()
