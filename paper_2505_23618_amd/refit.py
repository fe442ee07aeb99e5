"""Differentiable adjusted transform (fp32) for refitting the band angles.

``AdjustedTransformFn`` wraps the library's Givens-band forward and backward
kernels (``ta_givens_fwd`` / ``ta_givens_bwd``) as a torch.autograd.Function:
y = B A(theta) x for a batch of vectors x[m, n], with gradients for x and the
angles theta.  The binding only marshals pointers and the stream; the
forward, the adjoint and the angle-gradient reduction run in HIP kernels.

``refit_loss`` is the refit objective: squared distance of the first P basis
functions of H = B A(theta) to the exact DST-7 (rows of H obtained by
transforming the unit vectors with the same kernel) plus lam times the
fraction of the data's energy outside the first P coefficients.
"""

from __future__ import annotations

import ctypes
import math

import torch

from . import DCT2, DST3, _check, _stream_handle, lib


def n_angles(n: int, taps: int) -> int:
    return sum((n - 2 - (l & 1)) // 2 + 1 for l in range(taps // 2))


class AdjustedTransformFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, tctx, base=DCT2, taps=4):
        if x.dtype != torch.float32 or theta.dtype != torch.float32 or not x.is_cuda:
            raise TypeError("expected fp32 GPU tensors")
        x = x.contiguous()
        theta = theta.contiguous()
        m, n = x.shape
        y = torch.empty_like(x)
        _check(lib().ta_givens_fwd(tctx._h, base, n, taps, ctypes.c_void_p(theta.data_ptr()), m,
                                   ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   _stream_handle(None)))
        ctx.save_for_backward(x, theta)
        ctx.tctx, ctx.base, ctx.taps = tctx, base, taps
        return y

    @staticmethod
    def backward(ctx, gy):
        x, theta = ctx.saved_tensors
        gy = gy.contiguous()
        m, n = x.shape
        gx = torch.empty_like(x)
        gth = torch.empty_like(theta)
        nbytes = ctypes.c_int64()
        _check(lib().ta_givens_workspace(m, ctypes.byref(nbytes)))
        ws = torch.empty(max(nbytes.value, 4), dtype=torch.uint8, device=x.device)
        _check(lib().ta_givens_bwd(ctx.tctx._h, ctx.base, n, ctx.taps, ctypes.c_void_p(theta.data_ptr()), m,
                                   ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                   ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gth.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()), _stream_handle(None)))
        return gx, gth, None, None, None


def adjusted(x, theta, tctx, base=DCT2, taps=4):
    return AdjustedTransformFn.apply(x, theta, tctx, base, taps)


def dst7_rows(n: int, device) -> torch.Tensor:
    """Exact orthonormal DST-7 rows (the target of the fit)."""
    k = torch.arange(n, dtype=torch.float64)[:, None]
    i = torch.arange(n, dtype=torch.float64)[None, :]
    d = math.sqrt(4.0 / (2 * n + 1)) * torch.sin(math.pi * (2 * k + 1) * (i + 1) / (2 * n + 1))
    return d.to(device=device, dtype=torch.float32)


def refit_loss(x, theta, tctx, base=DCT2, taps=4, p=8, lam=1.0):
    """Basis term + lam * energy-compaction term (see the module docstring)."""
    n = x.shape[1]
    eye = torch.eye(n, device=x.device, dtype=torch.float32)
    ht = adjusted(eye, theta, tctx, base, taps)          # row j = H e_j = column j of H
    h = ht.t()
    d = dst7_rows(n, x.device)
    basis = ((h[:p] - d[:p]) ** 2).sum()
    y = adjusted(x, theta, tctx, base, taps)
    energy = lam * (1.0 - (y[:, :p] ** 2).sum() / (x ** 2).sum())
    return basis + energy, basis, energy
