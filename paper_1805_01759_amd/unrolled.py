"""Differentiable unrolled fixed-step map (K iterations of Eqs. (11)-(12) of
arXiv 1805.01759 with a constant step) as a torch.autograd.Function.

Forward and backward run in libl1ls.so (l1ls_unrolled_forward / _backward);
this module only allocates the tape and workspace and marshals pointers.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .api import _ptr, _stream


def _aligned_bytes(nbytes: int, device) -> torch.Tensor:
    buf = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + max(int(nbytes), 256)]


class UnrolledFISTA(torch.autograd.Function):
    """X_K = map(B, lambda, xi); gradients for B (complex), lambda and xi."""

    @staticmethod
    def forward(ctx, B, lam, xi, s, alpha: float, K: int, ckpt: int):
        L = _lib.load()
        B = B.contiguous()
        xi32 = xi.detach().to(torch.float32).contiguous()
        s32 = s.detach().to(torch.float32).contiguous()
        n, l, p = xi32.numel(), s32.numel(), B.shape[0]
        lam_f = float(lam)
        sz = ctypes.c_size_t(0)
        _lib.check(L.l1ls_unrolled_tape_size(n, l, p, K, ckpt, ctypes.byref(sz)), "tape size")
        tape = _aligned_bytes(sz.value, B.device)
        X = torch.empty((p, l), dtype=torch.complex64, device=B.device)
        _lib.check(L.l1ls_unrolled_forward(n, l, p, _ptr(xi32), _ptr(s32), _ptr(B), lam_f,
                                           float(alpha), K, ckpt, _ptr(X), _ptr(tape), tape.numel(),
                                           _stream()), "l1ls_unrolled_forward")
        ctx.save_for_backward(B, xi32, s32, tape)
        ctx.meta = (lam_f, float(alpha), int(K), int(ckpt), torch.is_tensor(lam))
        return X

    @staticmethod
    def backward(ctx, dX):
        L = _lib.load()
        B, xi32, s32, tape = ctx.saved_tensors
        lam_f, alpha, K, ckpt, lam_is_tensor = ctx.meta
        n, l, p = xi32.numel(), s32.numel(), B.shape[0]
        dX = dX.to(torch.complex64).contiguous()
        sz = ctypes.c_size_t(0)
        _lib.check(L.l1ls_unrolled_backward_ws_size(n, l, p, K, ckpt, ctypes.byref(sz)), "ws size")
        ws = _aligned_bytes(sz.value, B.device)
        dB = torch.empty_like(B)
        dlam = torch.empty(1, dtype=torch.float32, device=B.device)
        dxi = torch.empty(n, dtype=torch.float32, device=B.device)
        _lib.check(L.l1ls_unrolled_backward(n, l, p, _ptr(xi32), _ptr(s32), _ptr(B), lam_f, alpha,
                                            K, ckpt, _ptr(tape), tape.numel(), _ptr(dX), _ptr(dB),
                                            _ptr(dlam), _ptr(dxi), _ptr(ws), ws.numel(), _stream()),
                   "l1ls_unrolled_backward")
        return dB, (dlam[0] if lam_is_tensor else None), dxi, None, None, None, None


def unrolled(B, lam, xi, s, alpha: float, K: int = 200, ckpt: int = 20):
    return UnrolledFISTA.apply(B, lam, xi, s, alpha, K, ckpt)
