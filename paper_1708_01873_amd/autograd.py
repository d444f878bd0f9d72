"""Differentiable bit-reversed permutation for PyTorch.

``BitRev.apply(x)`` permutes the last dimension of ``x`` (length 2^k) row by
row with the library's ``bitrev_rows`` kernel.  The permutation matrix P
satisfies P^T = P because rev_k(rev_k(i)) = i (arXiv:1708.01873,
Introduction), so the backward applies the same kernel to the incoming
gradient: dL/dx = P^T g = P g.  Nothing is saved for backward.
"""
from __future__ import annotations

import torch

from . import bitrev_rows


def _log2_last(x: torch.Tensor) -> int:
    if x.dim() == 0:
        raise ValueError("BitRev needs at least one dimension")
    n = x.shape[-1]
    k = int(n).bit_length() - 1
    if n <= 0 or (1 << k) != n:
        raise ValueError("last dimension %d is not a power of two" % n)
    return k


class BitRev(torch.autograd.Function):
    """y[..., rev(j)] = x[..., j]; backward: the same permutation of grad."""

    @staticmethod
    def forward(ctx, x: torch.Tensor) -> torch.Tensor:
        k = _log2_last(x)
        x = x.contiguous()
        y = torch.empty_like(x)
        if x.numel():
            bitrev_rows(x, y, k)
        return y

    @staticmethod
    def backward(ctx, grad: torch.Tensor) -> torch.Tensor:
        # The adjoint is the permutation itself; applying it through BitRev
        # keeps higher-order gradients available.
        return BitRev.apply(grad)


def bitrev(x: torch.Tensor) -> torch.Tensor:
    """Differentiable bit-reversed permutation of the last dimension."""
    return BitRev.apply(x)
