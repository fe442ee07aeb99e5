"""FP64 separable 2-D adjusted transforms (test infrastructure).

Y = H_v X H_h^T (forward: each row of X transformed by the horizontal H_h,
each column by the vertical H_v) and X = H_v^T Y H_h (inverse), with every H
built as C B A (eq. 1) and the DCT-8 flip S H R (eq. 3) by
``oracle.adjust.adjusted``; section 2.2 applies the adjustment along both
directions of the block (W x B and B x H strips for the sub-block case), which
is exactly what the separable product does.

Pins (tests/test_oracle_fp.py): orthogonality of every H so inverse(forward)
returns X to 1e-12; with no adjustment the 2-D DCT-2 equals
scipy.fft.dctn(type=2, norm="ortho"); the separable product equals the
Kronecker-product form (H_v kron H_h) vec(X).
"""

from __future__ import annotations

import numpy as np

from . import adjust
from .fixed import Axis


def axis_matrix(ax: Axis, n: int) -> np.ndarray:
    if ax.adj == "band":
        return adjust.adjusted(ax.base, n, a=np.asarray(ax.a_f), flip=ax.flip)
    if ax.adj == "post":
        return adjust.adjusted(ax.base, n, c=adjust.post_matrix(n, np.asarray(ax.q_f)), flip=ax.flip)
    return adjust.adjusted(ax.base, n, flip=ax.flip)


def fwd2d(x: np.ndarray, ax_h: Axis, ax_v: Axis) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    hh = axis_matrix(ax_h, x.shape[-1])
    hv = axis_matrix(ax_v, x.shape[-2])
    return np.einsum("ij,bjk,lk->bil", hv, x, hh)


def inv2d(y: np.ndarray, ax_h: Axis, ax_v: Axis) -> np.ndarray:
    y = np.asarray(y, dtype=np.float64)
    hh = axis_matrix(ax_h, y.shape[-1])
    hv = axis_matrix(ax_v, y.shape[-2])
    return np.einsum("ji,bjk,kl->bil", hv, y, hh)
