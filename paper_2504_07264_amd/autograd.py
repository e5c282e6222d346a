"""Autograd wrapper: the split-format DFT as a differentiable op.

The forward is eq. (5) of the paper, (yr, yi) = E_2N (xr, xi) with
E_2N = [[C, S], [-S, C]].  It is linear, so its vector-Jacobian product is
the transpose E_2N^T = [[C, -S], [S, C]] (C and S are symmetric) applied to
the incoming gradient, computed by the library's adjoint kernel.  Nothing is
saved for the backward.
"""
from __future__ import annotations

import torch

from .binding import cached_plan


def _operand(t: torch.Tensor) -> torch.Tensor:
    """Contiguous and 16-byte aligned (the library's requirement): a view that
    starts inside an allocation is copied."""
    t = t.contiguous()
    return t if t.data_ptr() % 16 == 0 else t.clone()


class SplitDFTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xr: torch.Tensor, xi: torch.Tensor):
        if xr.shape != xi.shape:
            raise ValueError("xr and xi differ in shape")
        n = xr.shape[-1]
        batch = xr.numel() // n
        ctx.meta = (n, batch, xr.device, xr.shape)
        p = cached_plan(n, batch, xr.device)
        yr, yi = p.exec(_operand(xr), _operand(xi))
        return yr.view(xr.shape), yi.view(xr.shape)

    @staticmethod
    def backward(ctx, gyr, gyi):
        n, batch, device, shape = ctx.meta
        if gyr is None:
            gyr = torch.zeros(shape, dtype=torch.float32, device=device)
        if gyi is None:
            gyi = torch.zeros(shape, dtype=torch.float32, device=device)
        p = cached_plan(n, batch, device)
        gxr, gxi = p.adjoint(_operand(gyr), _operand(gyi))
        return gxr.view(shape), gxi.view(shape)


def split_dft_autograd(xr: torch.Tensor, xi: torch.Tensor):
    """Differentiable forward split-format DFT of the rows of (xr, xi)."""
    return SplitDFTFunction.apply(xr, xi)
