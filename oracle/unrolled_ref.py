"""Plain-PyTorch complex128 CPU reference of the unrolled fixed-step map.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  The forward pass is
Eqs. (11)-(12) of arXiv 1805.01759 with a constant step alpha, no backtracking
and no monotone test, K iterations from x^0 = x^{-1} = 0; A is built from the
spatial frequencies xi_n of Eq. (2) as A[n, l] = exp(-j 2 pi xi_n s_l).  The
gradients of loss = sum |X_K - X_true|^2 with respect to B, lambda and xi come
from torch autograd (complex gradients follow PyTorch's convention
dL/dRe + j dL/dIm).
"""
from __future__ import annotations

import math

import torch


def build_A(xi: torch.Tensor, s: torch.Tensor) -> torch.Tensor:
    phase = -2.0 * math.pi * torch.outer(xi, s)
    return torch.polar(torch.ones_like(phase), phase)


def prox(v: torch.Tensor, tau: torch.Tensor) -> torch.Tensor:
    """S_tau(v) = v max(0, 1 - tau/|v|); |v| <= tau -> 0 (Eq. (10), complex form)."""
    mag = v.abs()
    keep = mag > tau
    safe = torch.where(keep, mag, torch.ones_like(mag))
    scale = torch.where(keep, 1.0 - tau / safe, torch.zeros_like(mag))
    return v * scale


def unrolled(xi, s, B, lam, alpha: float, K: int):
    """X_K for every pixel row of B (complex128 tensors; lam a 0-d real tensor)."""
    A = build_A(xi, s)
    P, L = B.shape[0], s.shape[0]
    x = torch.zeros(P, L, dtype=torch.complex128)
    xprev = torch.zeros_like(x)
    for k in range(1, K + 1):
        beta = max(0.0, (k - 2) / (k + 1))
        y = x + beta * (x - xprev)
        r = y @ A.transpose(0, 1) - B           # (P, N): A y - b per pixel
        g = 2.0 * (r @ A.conj())                # (P, L): 2 A^H r per pixel
        xprev = x
        x = prox(y - alpha * g, alpha * lam)
    return x


def loss_and_grads(xi, s, B, lam, alpha, K, Xtrue):
    """loss = sum |X_K - X_true|^2 and its gradients (dB complex, dlam, dxi)."""
    xi = xi.clone().detach().to(torch.float64).requires_grad_(True)
    B = B.clone().detach().to(torch.complex128).requires_grad_(True)
    lam = torch.as_tensor(lam, dtype=torch.float64).clone().detach().requires_grad_(True)
    X = unrolled(xi, s.to(torch.float64), B, lam, alpha, K)
    loss = (X - Xtrue.to(torch.complex128)).abs().pow(2).sum()
    loss.backward()
    return loss.detach(), X.detach(), B.grad.detach(), lam.grad.detach(), xi.grad.detach()
