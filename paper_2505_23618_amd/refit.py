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


_CONSTS = {}


def _consts(n: int, device):
    """The identity and the exact DST-7 rows of size n on `device`, built once
    (a step then launches no host-to-device copy)."""
    key = (n, str(device))
    if key not in _CONSTS:
        _CONSTS[key] = (torch.eye(n, device=device, dtype=torch.float32), dst7_rows(n, device))
    return _CONSTS[key]


def refit_loss(x, theta, tctx, base=DCT2, taps=4, p=8, lam=1.0):
    """Basis term + lam * energy-compaction term (see the module docstring)."""
    n = x.shape[1]
    eye, d = _consts(n, x.device)
    ht = adjusted(eye, theta, tctx, base, taps)          # row j = H e_j = column j of H
    h = ht.t()
    basis = ((h[:p] - d[:p]) ** 2).sum()
    y = adjusted(x, theta, tctx, base, taps)
    energy = lam * (1.0 - (y[:, :p] ** 2).sum() / (x ** 2).sum())
    return basis + energy, basis, energy


class GraphedRefitStep:
    """One refit step (refit_loss forward and backward) captured once in a HIP
    graph and replayed: replay() recomputes the loss terms and theta.grad for
    the current contents of x and theta, which must stay the same tensors
    (update them in place, and leave theta.grad in place: the graph writes
    that tensor).  Launch overhead is what dominates an eager step on a
    cache-resident batch; the replay issues the same kernels as one graph."""

    def __init__(self, x, theta, tctx, base=DCT2, taps=4, p=8, lam=1.0, warmup=2):
        self.x, self.theta = x, theta
        args = (tctx, base, taps, p, lam)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                theta.grad = None
                # no reference to the warm-up's loss terms survives the loop, so
                # the capture does not find their autograd graph (and the
                # angles' gradient accumulator made on this stream) alive
                refit_loss(x, theta, *args)[0].backward()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        theta.grad = None
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.loss, self.basis, self.energy = refit_loss(x, theta, *args)
            self.loss.backward()
        self.grad = theta.grad

    def replay(self):
        self.graph.replay()
        return self.loss

