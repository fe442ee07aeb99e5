"""Backward of the separable 2-D adjusted transform over a list of blocks,
FP64 (test infrastructure; never imported by the product path).

Forward, per block b (section 2.2, eq. 1, eq. 3):
    Y_b = H_v X_b H_h^T,   H = S^f B A R^f  (band)  or  S^f C B R^f  (sub-block),
f = 1 for a DCT-8 axis built from a DST-7 design.  The adjustment of one
parameter set is parametrised by angles (section 2: orthogonality through
sequential sets of parallel Givens rotations):
    band      A(theta) = G_{L-1} ... G_0             (oracle.adjust.band_matrix)
    sub-block C = blkdiag(Q, I),  Q = Q0 R(phi)     (oracle.adjust.rotation_product)
Given G_Y = dL/dY for every block, the backward returns
    dL/dX_b = H_v^T G_Y H_h                                    (the adjoint)
    dL/dH_h += G_Y^T H_v X_b,   dL/dH_v += G_Y H_h X_b^T       (per use of the set)
and, through H = S^f B A R^f, dL/dA = B^T S^f (dL/dH) R^f; through
H = S^f C B R^f, dL/dC = S^f (dL/dH) (B R^f)^T whose top-left B x B block is
dL/dQ; then the angle gradient by the chain rule through the rotations
(oracle.adjust.band_grad, and rotation_product_grad with Q0^T dL/dQ).

Pins (tests/test_oracle_blockgrad.py): the angle gradient against FP64
central differences of L(theta) = sum_b <G_Y, Y_b(theta)>, and dL/dX against
central differences in X; a set used by no axis has a zero gradient; with
both axes of a square block on the same set the gradient is the sum of the
two one-axis gradients.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import adjust
from . import transforms as T


@dataclass
class AngleSet:
    """An angle-parametrised adjustment of size n: a band of `taps` taps
    (theta, taps // 2 layers) or a b x b sub-block Q0 R(phi)."""
    kind: str          # "band" or "post"
    n: int
    angles: np.ndarray
    taps: int = 0
    b: int = 0
    q0: np.ndarray | None = None

    def matrix(self) -> np.ndarray:
        """A (band, n x n) or Q (sub-block, b x b)."""
        if self.kind == "band":
            return adjust.band_matrix(self.n, self.taps // 2, self.angles)
        q0 = np.eye(self.b) if self.q0 is None else np.asarray(self.q0, np.float64)
        return q0 @ adjust.rotation_product(self.b, self.angles)


@dataclass
class AxisUse:
    """One axis: its base and flip, and whether its adjustment is the
    angle set (param=True) or fixed (adjustment matrices a / q given)."""
    base: str
    adj: str = "none"
    flip: bool = False
    param: bool = False
    a: np.ndarray | None = None
    q: np.ndarray | None = None


def axis_matrix(ax: AxisUse, n: int, aset: AngleSet | None) -> np.ndarray:
    """H of one axis (eq. 1 and the flip of eq. 3)."""
    h = T.matrix(ax.base, n)
    if ax.adj == "band":
        a = aset.matrix() if ax.param else np.asarray(ax.a)
        h = h @ a
    elif ax.adj == "post":
        q = aset.matrix() if ax.param else np.asarray(ax.q)
        h = adjust.post_matrix(n, q) @ h
    if ax.flip:
        h = T.signs(n) @ h @ T.reversal(n)
    return h


def forward(blocks, axes, aset):
    """Y_b = H_v X_b H_h^T for a list of blocks X_b [H, W] with axes
    (h, v) per block."""
    out = []
    for x, (ah, av) in zip(blocks, axes):
        hv = axis_matrix(av, x.shape[0], aset)
        hh = axis_matrix(ah, x.shape[1], aset)
        out.append(hv @ np.asarray(x, np.float64) @ hh.T)
    return out


def _matrix_grad(ax: AxisUse, n: int, gh: np.ndarray) -> np.ndarray:
    """dL/dA (band) or dL/dQ (sub-block) from dL/dH of one axis."""
    r = T.reversal(n) if ax.flip else np.eye(n)
    s = T.signs(n) if ax.flip else np.eye(n)
    b = T.matrix(ax.base, n)
    if ax.adj == "band":
        return b.T @ s @ gh @ r                      # H = S B A R
    gc = s @ gh @ (b @ r).T                          # H = S C B R
    return gc


def backward(blocks, axes, gys, aset: AngleSet):
    """(dL/dX per block, dL/d angles) for dL/dY = gys."""
    gxs = []
    gm = np.zeros((aset.n, aset.n) if aset.kind == "band" else (aset.b, aset.b))
    for x, (ah, av), gy in zip(blocks, axes, gys):
        x = np.asarray(x, np.float64)
        gy = np.asarray(gy, np.float64)
        hv = axis_matrix(av, x.shape[0], aset)
        hh = axis_matrix(ah, x.shape[1], aset)
        gxs.append(hv.T @ gy @ hh)
        if ah.param:
            m = _matrix_grad(ah, x.shape[1], gy.T @ hv @ x)
            gm += m if aset.kind == "band" else m[:aset.b, :aset.b]
        if av.param:
            m = _matrix_grad(av, x.shape[0], gy @ hh @ x.T)
            gm += m if aset.kind == "band" else m[:aset.b, :aset.b]
    if aset.kind == "band":
        gth = adjust.band_grad(aset.n, aset.taps // 2, aset.angles, gm)
    else:
        q0 = np.eye(aset.b) if aset.q0 is None else np.asarray(aset.q0, np.float64)
        gth = adjust.rotation_product_grad(aset.b, aset.angles, q0.T @ gm)
    return gxs, gth
