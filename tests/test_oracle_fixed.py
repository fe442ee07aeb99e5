"""Pins of oracle.fixed: integer tables, error bounds, closed forms, roundtrip."""

import numpy as np
import pytest

import synth
from oracle import fixed as F
from oracle import fp as P
from oracle import transforms as T
from oracle.adjust import round_half_away
from tests import cfgs

SIZES = [4, 8, 16, 32, 64]


def test_rs_and_clip_worked_values():
    # RS(v, s) = floor((v + 2^(s-1)) / 2^s): half rounds up (towards +inf)
    v = np.array([5, -5, 6, -6, 7, -7, 0, 1, -1])
    assert F.rs(v, 1).tolist() == [3, -2, 3, -3, 4, -3, 0, 1, 0]
    assert F.rs(v, 2).tolist() == [1, -1, 2, -1, 2, -2, 0, 0, 0]
    assert F.rs(v, 0).tolist() == v.tolist()
    assert F.clip16(np.array([40000, -40000, 5])).tolist() == [32767, -32768, 5]


@pytest.mark.parametrize("n", SIZES)
def test_integer_table_invariants(n):
    c2 = F.int_table("C2", n)
    # DC row is exactly 2^m: 2^m sqrt(N) sqrt(2/N) / sqrt2 = 2^m
    assert (c2[0] == 256).all()
    # row symmetry: T[k][N-1-n] = (-1)^k T[k][n]
    for k in range(n):
        assert (c2[k, ::-1] == ((-1) ** k) * c2[k]).all()
    # nesting: even rows of size N are the rows of size N/2 (left half)
    if n > 4:
        half = F.int_table("C2", n // 2)
        assert (c2[0::2, : n // 2] == half).all()
    # magnitude bound 2^m sqrt2 = 362.04; the largest entry is row 1, column 0
    assert np.abs(c2).max() == c2[1, 0] <= 362
    # derived DST-2/DST-3 equal their own directly rounded formulas
    for kind in ("S2", "S3", "C3"):
        direct = round_half_away(256.0 * np.sqrt(n) * T.matrix(kind, n))
        assert (F.int_table(kind, n) == direct).all(), kind
    # DCT-8 integer table equals S DST-7_int R (eq. 3 on the rounded tables)
    s, r = T.signs(n).astype(np.int64), T.reversal(n).astype(np.int64)
    assert (F.int_table("C8", n) == s @ F.int_table("S7", n) @ r).all()


def _rational_and_bound(x, ax_h, ax_v, bd, m, a, inverse=False):
    """Un-rounded product of the integer stages (exact rational, in FP64) and
    the worst-case propagated rounding error (0.5 LSB per stage, amplified by
    the later stages' absolute row sums)."""
    nb, h, w = x.shape
    s1, s2, s3, s4 = F.shifts(int(np.log2(w)), int(np.log2(h)), bd, m)
    sh, sv = F.forward_stages(ax_h, w, m, a), F.forward_stages(ax_v, h, m, a)
    if inverse:
        seq = [("v", st.T, s3 if r == "core" else a) for st, r in reversed(sv)] + \
              [("h", st.T, s4 if r == "core" else a) for st, r in reversed(sh)]
    else:
        seq = [("h", st, s1 if r == "core" else a) for st, r in sh] + \
              [("v", st, s2 if r == "core" else a) for st, r in sv]
    v = x.astype(np.float64)
    err = 0.0
    for axis, mat, s in seq:
        mf = mat.astype(np.float64) / (2.0 ** s)
        if axis == "h":
            v = np.einsum("bij,kj->bik", v, mf)
        else:
            v = np.einsum("kj,bji->bki", mf, v)
        err = np.abs(mf).sum(axis=1).max() * err + 0.5
    return v, err


@pytest.mark.parametrize("which", ["cfg1", "cfg2", "cfg3", "c2plain", "s7direct"])
def test_fixed_equals_rational_within_rounding_bound(params, which, rng):
    if which == "cfg1":
        ax_h, ax_v = cfgs.cfg1(params); n = 16
    elif which == "cfg2":
        ax_h, ax_v = cfgs.cfg2(params); n = 32
    elif which == "cfg3":
        ax_h, ax_v = cfgs.cfg3(params); n = 64
    elif which == "c2plain":
        ax_h = ax_v = cfgs.plain_axis("C2"); n = 32
    else:
        ax_h = ax_v = cfgs.plain_axis("S7"); n = 16
    x = synth.ar1_blocks(24, n, n, 0.95, 16.0, seed=7)
    y = F.fwd2d(x, ax_h, ax_v)
    ref, bound = _rational_and_bound(x, ax_h, ax_v, 8, 8, 10)
    assert np.abs(ref).max() < 32767          # no clipping on this data
    d = y - ref
    assert np.abs(d).max() <= bound + 1e-9
    assert abs(d.mean()) < 0.1                 # round-to-nearest, unbiased
    xi = F.inv2d(y, ax_h, ax_v)
    ref, bound = _rational_and_bound(y, ax_h, ax_v, 8, 8, 10, inverse=True)
    assert np.abs(xi - ref).max() <= bound + 1e-9


@pytest.mark.parametrize("which", ["cfg1", "cfg2", "cfg3"])
def test_fixed_tracks_fp64_transform(params, which):
    # forward gain 2^(15-bd)/sqrt(WH): the integer result is the FP64 adjusted
    # transform scaled, up to table/parameter quantisation
    ax_h, ax_v = {"cfg1": cfgs.cfg1, "cfg2": cfgs.cfg2, "cfg3": cfgs.cfg3}[which](params)
    n = {"cfg1": 16, "cfg2": 32, "cfg3": 64}[which]
    x = synth.ar1_blocks(16, n, n, 0.95, 16.0, seed=3)
    y = F.fwd2d(x, ax_h, ax_v)
    g = 2.0 ** (15 - 8) / n
    yf = g * P.fwd2d(x, ax_h, ax_v)
    rel = np.abs(y - yf).max() / np.abs(yf).max()
    assert rel < 5e-3


@pytest.mark.parametrize("n", SIZES)
def test_constant_block_dct2_closed_form(n):
    # a constant block c through the plain 2-D DCT-2 gives only a DC value;
    # row pass: RS(N * c * 2^m, s1); column pass: RS(N * dc1 * 2^m, s2)
    c = 200
    x = np.full((1, n, n), c, np.int16)
    ax = cfgs.plain_axis("C2")
    y = F.fwd2d(x, ax, ax)
    l2 = int(np.log2(n))
    s1, s2 = l2 + 8 + 8 - 15, l2 + 8
    dc1 = (n * c * 256 + (1 << (s1 - 1))) >> s1
    dc = (n * dc1 * 256 + (1 << (s2 - 1))) >> s2
    assert y[0, 0, 0] == dc
    # other outputs vanish up to the rounding of the even rows' sums
    rest = y.copy()
    rest[0, 0, 0] = 0
    assert np.abs(rest).max() <= 1


@pytest.mark.parametrize("which", ["cfg1", "cfg2", "cfg3"])
def test_roundtrip_statistics(params, which):
    ax_h, ax_v = {"cfg1": cfgs.cfg1, "cfg2": cfgs.cfg2, "cfg3": cfgs.cfg3}[which](params)
    n = {"cfg1": 16, "cfg2": 32, "cfg3": 64}[which]
    x = synth.ar1_blocks(32, n, n, 0.95, 16.0, seed=11)
    xr = F.inv2d(F.fwd2d(x, ax_h, ax_v), ax_h, ax_v)
    err = np.abs(xr - x)
    assert err.max() <= 8
    assert err.mean() < 0.5


@pytest.mark.parametrize("kind", ["pos", "neg", "checker", "full16", "extreme16"])
def test_adversarial_inputs_stay_in_range_and_headroom(params, kind):
    # the headroom assertion inside the oracle must hold for any int16 input
    ax_h, ax_v = cfgs.cfg2(params)
    x = synth.adversarial_blocks(32, 32, kind)
    y = F.fwd2d(x, ax_h, ax_v)
    assert y.min() >= -32768 and y.max() <= 32767
    z = F.inv2d(x, ax_h, ax_v)
    assert z.min() >= -32768 and z.max() <= 32767


def test_flip_band_equals_flipped_matrices(params):
    # adjusted DCT-8 by flip: integer stages compose to S (B_int A_int) R
    ax = cfgs.band_axis(params, "S3", 16, 4, flip=True)
    st = F.forward_stages(ax, 16, 8, 10)
    ax0 = cfgs.band_axis(params, "S3", 16, 4, flip=False)
    st0 = F.forward_stages(ax0, 16, 8, 10)
    s, r = T.signs(16).astype(np.int64), T.reversal(16).astype(np.int64)
    assert (st[1][0] @ st[0][0] == s @ st0[1][0] @ st0[0][0] @ r).all()


def test_single_pass_headroom_holds_for_all_int16():
    # worst case: every input at +-32768 aligned with the row signs
    for n in SIZES:
        for kind in ("C2", "C3", "S7"):
            t = F.int_table(kind, n)
            assert int(np.abs(t).sum(axis=1).max()) * 32768 < (1 << 31)


def _rs(v, s):
    return (v + (1 << (s - 1))) >> s if s > 0 else v


@pytest.mark.parametrize("bd", [8, 10])
@pytest.mark.parametrize("lw,lh", [(2, 2), (3, 5), (5, 5), (6, 6), (6, 3)])
def test_dc_only_inverse_dct2_closed_form(bd, lw, lh):
    """A block whose only non-zero coefficient is the DC value c, through the
    plain inverse 2-D DCT-2, worked out by hand.  Every entry of the integer
    DC row is 2^m = 256, so the column pass (inverse first, shift m + 1 = 9)
    turns column 0 into the constant RS(256 c, 9) and leaves the other columns
    zero; the row pass (shift m + 14 - bd) then spreads that value over the
    row: every residual equals RS(256 RS(256 c, 9), 22 - bd).  The two
    shifts are pinned one by one: the same chain with one bit moved from
    one stage to the other differs from it for some c in the range."""
    w, h = 1 << lw, 1 << lh
    cs = np.arange(-4000, 4001, 7)
    y = np.zeros((len(cs), h, w), np.int64)
    y[:, 0, 0] = cs
    ax = cfgs.plain_axis("C2")
    x = F.inv2d(y, ax, ax, bd=bd)
    chain = [_rs(256 * _rs(256 * int(c), 9), 22 - bd) for c in cs]
    assert (x == np.asarray(chain)[:, None, None]).all()
    for s_col, s_row in ((10, 21 - bd), (8, 23 - bd)):
        moved = [_rs(256 * _rs(256 * int(c), s_col), s_row) for c in cs]
        assert moved != chain, (s_col, s_row)


@pytest.mark.parametrize("bd", [8, 10])
def test_dc_only_forward_then_inverse_chain(bd):
    """Constant residual blocks c: the forward DC (rows shift log2 W + bd - 7,
    columns log2 H + 8) followed by the inverse chain above, all by hand."""
    lw, lh = 4, 3
    w, h = 1 << lw, 1 << lh
    cs = np.arange(-255, 256, 3)
    x = np.broadcast_to(cs[:, None, None], (len(cs), h, w)).astype(np.int64)
    ax = cfgs.plain_axis("C2")
    y = F.fwd2d(x, ax, ax, bd=bd)
    dc = [_rs(h * 256 * _rs(w * 256 * int(c), lw + bd - 7), lh + 8) for c in cs]
    assert (y[:, 0, 0] == np.asarray(dc)).all()
    xr = F.inv2d(np.where(np.arange(h * w).reshape(1, h, w) == 0, y, 0), ax, ax, bd=bd)
    back = [_rs(256 * _rs(256 * d, 9), 22 - bd) for d in dc]
    assert (xr == np.asarray(back)[:, None, None]).all()


# ---------------------------------------------------------------------------
# The same fixed-point reading written out here, independently of
# oracle.fixed's stage and shift helpers: integer tables rounded directly from
# the FP64 formulas, the stage order of each axis kind, and the core shifts.
# ---------------------------------------------------------------------------
def _int_mat(kind, n, m=8):
    return round_half_away((2.0 ** m) * np.sqrt(n) * T.matrix(kind, n)).astype(np.float64)


def _stages_written_out(ax, n, a, m=8):
    """Forward stages of one axis as (matrix, 'core' | 'adj'): with f the DCT-8
    flip, none = [S^f B R^f]; band = [A R^f (a), S^f B (core)];
    post = [S^f B R^f (core), blkdiag(S^f Q S^f, 2^a I) (a)]."""
    b = _int_mat(ax.base, n, m)
    idx = np.arange(n)
    rev = np.eye(n)[::-1] if ax.flip else np.eye(n)
    sgn = np.diag((-1.0) ** idx) if ax.flip else np.eye(n)
    if ax.adj == "none":
        return [(sgn @ b @ rev, "core")]
    if ax.adj == "band":
        return [(np.asarray(ax.a_int, np.float64) @ rev, "adj"), (sgn @ b, "core")]
    q = np.asarray(ax.q_int, np.float64)
    bb = q.shape[0]
    sq = np.diag((-1.0) ** np.arange(bb)) if ax.flip else np.eye(bb)
    c = (2.0 ** a) * np.eye(n)
    c[:bb, :bb] = sq @ q @ sq
    return [(sgn @ b @ rev, "core"), (c, "adj")]


def _rational_written_out(x, ax_h, ax_v, bd, a, inverse):
    nb, h, w = x.shape
    lw, lh, m = int(np.log2(w)), int(np.log2(h)), 8
    fwd_row, fwd_col = lw + bd + m - 15, lh + m           # forward: rows first
    inv_col, inv_row = m + 1, m + 14 - bd                  # inverse: columns first
    sh, sv = _stages_written_out(ax_h, w, a), _stages_written_out(ax_v, h, a)
    if inverse:
        seq = [("v", st.T, inv_col if r == "core" else a) for st, r in reversed(sv)] + \
              [("h", st.T, inv_row if r == "core" else a) for st, r in reversed(sh)]
    else:
        seq = [("h", st, fwd_row if r == "core" else a) for st, r in sh] + \
              [("v", st, fwd_col if r == "core" else a) for st, r in sv]
    v = x.astype(np.float64)
    err = 0.0
    for axis, mat, s in seq:
        mf = mat / (2.0 ** s)
        v = v @ mf.T if axis == "h" else np.einsum("kj,bji->bki", mf, v)
        err = np.abs(mf).sum(axis=1).max() * err + 0.5
    return v, err


@pytest.mark.parametrize("which", ["cfg1", "cfg2", "cfg2_flip", "cfg3", "post8", "s2_c8", "s7direct"])
@pytest.mark.parametrize("bd", [8, 10])
def test_fixed_within_bound_of_reading_written_out(params, which, bd):
    """The oracle's integers lie within the propagated rounding bound of the
    exact rational product of the stages as the reading states them (written
    out above, not taken from oracle.fixed), forward and inverse, with a
    tight bias check; so a stage in the wrong order, a missing flip or a
    shift off by one in any stage fails here."""
    if which == "cfg1":
        ax_h, ax_v = cfgs.cfg1(params); w = h = 16
    elif which == "cfg2":
        ax_h, ax_v = cfgs.cfg2(params); w = h = 32
    elif which == "cfg2_flip":
        ax_h = cfgs.band_axis(params, "S3", 32, 4, flip=True)
        ax_v = cfgs.band_axis(params, "S3", 16, 6)
        w, h = 32, 16
    elif which == "cfg3":
        ax_h, ax_v = cfgs.cfg3(params); w = h = 64
    elif which == "post8":
        ax_h, ax_v = cfgs.post_axis(params, 32, 8, flip=True), cfgs.post_axis(params, 16, 8); w, h = 32, 16
    elif which == "s2_c8":
        ax_h, ax_v = cfgs.plain_axis("S2"), cfgs.plain_axis("S7", flip=True); w, h = 8, 16
    else:
        ax_h = ax_v = cfgs.plain_axis("S7"); w = h = 16
    x = synth.ar1_blocks(24, h, w, 0.95, 16.0, seed=17)
    if bd == 10:
        x = x * 4
    y = F.fwd2d(x, ax_h, ax_v, bd=bd)
    ref, bound = _rational_written_out(x, ax_h, ax_v, bd, 10, inverse=False)
    assert np.abs(ref).max() < 32767
    d = y - ref
    assert np.abs(d).max() <= bound + 1e-9
    assert abs(d.mean()) < 0.1
    xi = F.inv2d(y, ax_h, ax_v, bd=bd)
    ref, bound = _rational_written_out(y, ax_h, ax_v, bd, 10, inverse=True)
    assert np.abs(xi - ref).max() <= bound + 1e-9
    assert abs((xi - ref).mean()) < 0.1
