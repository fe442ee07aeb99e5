"""Fixed-point separable 2-D adjusted transforms, dense int64 (test infrastructure).

The paper integrates the adjustments into the VTM-3.0 integer transforms
(section 3) but does not print that arithmetic.  Reading used here, in the
style of the VVC integer transforms, with integer-matrix precision m, bit depth
bd and adjustment precision a:

  integer tables   T_int = round_half_away(2^m sqrt(N) T) for DCT-2, DST-7,
                   DCT-8; DCT-3, DST-2, DST-3 are the section 2.1 relations
                   applied to the integer DCT-2 (transpose, R and S)
  adjustments      A_int = round_half_away(2^a A), Q_int = round_half_away(2^a Q)
  stage            v -> clip16(RS(M v, s)),  RS(v, s) = (v + 2^(s-1)) >> s
                   (arithmetic shift; RS(v, 0) = v), clip16 to [-32768, 32767]
  core shifts      forward: rows (first) s = log2 W + bd + m - 15,
                            columns s = log2 H + m;
                   inverse: columns (first) s = m + 1, rows s = m + 14 - bd
  adjust shifts    a

Per axis, the forward stage matrices (eq. 1 with one of A or C, and the DCT-8
flip S H R of eq. 3 / eq. 5):
  none            [S^f B_int R^f]
  band (pre)      [A_int R^f (a),  S^f B_int (core)]
  post            [S^f B_int R^f (core),  blkdiag(S^f Q_int S^f, 2^a I) (a)]
where ^f means "only when flipped".  The inverse applies the transposed stages
in reverse order.  Every product is evaluated as a dense int64 matrix product,
and the oracle asserts that the sum of the absolute values of the terms of
every dot product stays below 2^31, so that any int32 evaluation order
(butterfly, band taps, dot products) gives the same integers.

Pins (tests/test_oracle_fixed.py): integer-table invariants (row symmetry,
nesting of even rows, DC row exactly 2^m, derived DST-2/DST-3 tables equal to
their directly rounded formulas, DCT-8 table equal to S DST-7_int R); the 2-D
result equals the un-rounded rational product of the integer stages within the
propagated rounding bound, and is unbiased; constant blocks through the DCT-2
give the closed-form DC value; a DC-only coefficient block through the
inverse DCT-2 gives the hand-derived chain RS(256 RS(256 c, m + 1), m + 14 - bd)
at bit depths 8 and 10, which pins each inverse shift on its own (moving one
bit between the two stages changes the result); the 2-D result lies within
the rounding bound of the rational product of the stages as written out in
the test itself (tables rounded from the FP64 formulas, the stage order of
every axis kind with and without the flip, the four core shifts), forward
and inverse, unbiased; inverse(forward(x)) returns x within a few LSB.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import transforms as T
from .adjust import round_half_away

INT16_MIN, INT16_MAX = -32768, 32767


def rs(v: np.ndarray, s: int) -> np.ndarray:
    """RS(v, s) = (v + 2^(s-1)) >> s, arithmetic (flooring) shift; RS(v, 0) = v."""
    v = np.asarray(v, dtype=np.int64)
    if s == 0:
        return v.copy()
    return (v + (1 << (s - 1))) >> s


def clip16(v: np.ndarray) -> np.ndarray:
    return np.clip(v, INT16_MIN, INT16_MAX).astype(np.int64)


def int_table(kind: str, n: int, m: int = 8) -> np.ndarray:
    """Integer base tables (rows = basis vectors)."""
    if kind in ("C2", "S7", "C8"):
        return round_half_away((2.0 ** m) * np.sqrt(n) * T.matrix(kind, n))
    c2 = int_table("C2", n, m)
    r = T.reversal(n).astype(np.int64)
    s = T.signs(n).astype(np.int64)
    if kind == "C3":
        return c2.T.copy()
    if kind == "S2":
        return r @ c2 @ s
    if kind == "S3":
        return s @ c2.T @ r
    raise ValueError(kind)


@dataclass
class Axis:
    """One axis of a separable transform.

    base   one of C2, C3, S2, S3 (fast family) or S7, C8 (direct matrices)
    adj    "none", "band" (pre-adjustment A) or "post" (sub-block C)
    flip   DCT-8 version of a DST-7 design: H -> S H R (eq. 3, eq. 5)
    a_int  N x N integer band (scale 2^a) when adj == "band"
    q_int  B x B integer sub-block (scale 2^a) when adj == "post"
    a_f, q_f  the FP64 parameters (used by the FP64 path)
    """
    base: str
    adj: str = "none"
    flip: bool = False
    a_int: np.ndarray | None = None
    q_int: np.ndarray | None = None
    a_f: np.ndarray | None = None
    q_f: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def forward_stages(ax: Axis, n: int, m: int, a: int):
    """List of (integer matrix, role) with role in {"core", "adj"}."""
    b = int_table(ax.base, n, m)
    r = T.reversal(n).astype(np.int64)
    s = T.signs(n).astype(np.int64)
    one = np.eye(n, dtype=np.int64)
    rf = r if ax.flip else one
    sf = s if ax.flip else one
    if ax.adj == "none":
        return [(sf @ b @ rf, "core")]
    if ax.adj == "band":
        aint = np.asarray(ax.a_int, dtype=np.int64)
        return [(aint @ rf, "adj"), (sf @ b, "core")]
    if ax.adj == "post":
        q = np.asarray(ax.q_int, dtype=np.int64)
        bb = q.shape[0]
        c = (1 << a) * one
        sb = s[:bb, :bb] if ax.flip else np.eye(bb, dtype=np.int64)
        c[:bb, :bb] = sb @ q @ sb
        return [(sf @ b @ rf, "core"), (c, "adj")]
    raise ValueError(ax.adj)


def _apply(mat: np.ndarray, v: np.ndarray, s: int) -> np.ndarray:
    """clip16(RS(mat @ v, s)) over the first axis of v (columns are vectors)."""
    v = np.asarray(v, dtype=np.int64)
    bound = np.abs(mat) @ np.abs(v)
    assert int(bound.max(initial=0)) < (1 << 31), "int32 headroom violated"
    return clip16(rs(mat @ v, s))


def _pass(stages, v, s_core, a, inverse):
    seq = [(st.T, role) for st, role in reversed(stages)] if inverse else stages
    for mat, role in seq:
        v = _apply(mat, v, s_core if role == "core" else a)
    return v


def shifts(log2w: int, log2h: int, bd: int, m: int):
    """(forward row, forward column, inverse column, inverse row) core shifts."""
    return (log2w + bd + m - 15, log2h + m, m + 1, m + 14 - bd)


def fwd2d(x: np.ndarray, ax_h: Axis, ax_v: Axis, bd: int = 8, m: int = 8, a: int = 10) -> np.ndarray:
    """Forward 2-D fixed point of a batch x[nb, H, W] (int16 values): rows
    (horizontal transform) first, then columns.  Returns int64 [nb, H, W]."""
    x = np.asarray(x, dtype=np.int64)
    nb, h, w = x.shape
    s1, s2, _, _ = shifts(int(np.log2(w)), int(np.log2(h)), bd, m)
    sh = forward_stages(ax_h, w, m, a)
    sv = forward_stages(ax_v, h, m, a)
    # rows: each row is a vector of length W -> put W on the first axis
    z = x.transpose(2, 0, 1).reshape(w, nb * h)
    z = _pass(sh, z, s1, a, inverse=False)
    z = z.reshape(w, nb, h).transpose(1, 2, 0)               # nb, h, w
    # columns: vectors of length H
    y = z.transpose(1, 0, 2).reshape(h, nb * w)
    y = _pass(sv, y, s2, a, inverse=False)
    return y.reshape(h, nb, w).transpose(1, 0, 2).copy()


def inv2d(y: np.ndarray, ax_h: Axis, ax_v: Axis, bd: int = 8, m: int = 8, a: int = 10) -> np.ndarray:
    """Inverse 2-D fixed point: columns first (transposed vertical stages in
    reverse order), then rows."""
    y = np.asarray(y, dtype=np.int64)
    nb, h, w = y.shape
    _, _, s3, s4 = shifts(int(np.log2(w)), int(np.log2(h)), bd, m)
    sh = forward_stages(ax_h, w, m, a)
    sv = forward_stages(ax_v, h, m, a)
    z = y.transpose(1, 0, 2).reshape(h, nb * w)
    z = _pass(sv, z, s3, a, inverse=True)
    z = z.reshape(h, nb, w).transpose(1, 0, 2)                # nb, h, w
    x = z.transpose(2, 0, 1).reshape(w, nb * h)
    x = _pass(sh, x, s4, a, inverse=True)
    return x.reshape(w, nb, h).transpose(1, 2, 0).copy()


def pass1d(v: np.ndarray, ax: Axis, n: int, s_core: int, m: int = 8, a: int = 10,
           inverse: bool = False) -> np.ndarray:
    """One 1-D pass on column vectors v[n, k] (for the per-sample checks)."""
    return _pass(forward_stages(ax, n, m, a), np.asarray(v, np.int64), s_core, a, inverse)
