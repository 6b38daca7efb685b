"""torch.autograd.Function wrappers of the fused kernels.

The forward saves references to (u, F, M) only; no interpolation weights or
window statistics are stored.  The backward re-runs the fused adjoint kernel,
which recomputes the sampling weights and the statistics on the fly (the
paper's custom forward/backward kernels, Sec. "Composite Implicit Grid
Sampler" and App. "Fused LNCC" / "Implicit MI").  The upstream gradient is
handed to the kernel as a device pointer, so backward never synchronises
with the host.

Only the displacement is differentiable: the images are data (the sampler's
gradient with respect to the moving image is not needed on this path), and
asking for their gradient raises.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import ops


def _check_images(F, M):
    if F.requires_grad or M.requires_grad:
        raise NotImplementedError("gradients with respect to F or M are not provided; only u is differentiable")


class WarpLNCC(torch.autograd.Function):
    """loss = 1 - mean_ROI LNCC(F, M(x + u)) as a 0-dim tensor."""

    @staticmethod
    def forward(ctx, u, F, M, window: int = 5, eps: float = 1e-5, ants: bool = False, pad="border", roi=None):
        _check_images(F, M)
        loss = ops.warp_lncc_fwd(F, M, u, window=window, eps=eps, pad=pad, roi=roi)
        ctx.save_for_backward(u, F, M)
        ctx.cfg = (window, eps, ants, pad, roi)
        return loss.view(())

    @staticmethod
    def backward(ctx, g):
        u, F, M = ctx.saved_tensors
        window, eps, ants, pad, roi = ctx.cfg
        gs = g.detach().reshape(1).to(torch.float32).contiguous()
        grad_u, _ = ops.warp_lncc_bwd(F, M, u, window=window, eps=eps, ants=ants, pad=pad, roi=roi, grad_scale=gs,
                                      want_loss=False)
        return grad_u, None, None, None, None, None, None, None


class WarpMI(torch.autograd.Function):
    """loss = -MI(F, M(x + u)) with the Parzen B-spline histogram, 0-dim tensor."""

    @staticmethod
    def forward(ctx, u, F, M, bins: int = 32, pad="border", roi=None):
        _check_images(F, M)
        loss, state = ops.warp_mi_fwd(F, M, u, bins=bins, pad=pad, roi=roi)
        ctx.save_for_backward(u, F, M, state)
        ctx.cfg = (bins, pad, roi)
        return loss.view(())

    @staticmethod
    def backward(ctx, g):
        u, F, M, state = ctx.saved_tensors
        bins, pad, roi = ctx.cfg
        gs = g.detach().reshape(1).to(torch.float32).contiguous()
        grad_u = ops.warp_mi_bwd(F, M, u, state, bins=bins, pad=pad, roi=roi, grad_scale=gs)
        return grad_u, None, None, None, None, None


def lncc_loss(F: torch.Tensor, M: torch.Tensor, u: torch.Tensor, window: int = 5, eps: float = 1e-5,
              ants: bool = False, pad="border", roi=None) -> torch.Tensor:
    """Differentiable fused warp + LNCC loss (gradient flows to u)."""
    return WarpLNCC.apply(u, F, M, window, eps, ants, pad, roi)


def mi_loss(F: torch.Tensor, M: torch.Tensor, u: torch.Tensor, bins: int = 32, pad="border",
            roi: Optional[tuple] = None) -> torch.Tensor:
    """Differentiable fused warp + Parzen MI loss (-MI; gradient flows to u)."""
    return WarpMI.apply(u, F, M, bins, pad, roi)
