"""The integer tables the kernels compile in (csrc/tables_gen.h) meet the
bounds that make the packed kernels' scaled stages exact: with the table of
an N-point stage multiplied by 2^SC so that its shift becomes 16, every sum
of 2^SC * T * x over int16 inputs x must fit int32 and every rounded result
must fit int16 (the scaled stages apply no clamp)."""

import re
from pathlib import Path

import numpy as np
import pytest

TABLES = Path(__file__).resolve().parent.parent / "paper_2505_23618_amd" / "csrc" / "tables_gen.h"
XMAX, XMIN = 32767, -32768


def c2_64():
    text = TABLES.read_text()
    body = re.search(r"ta_c2_64\[64\]\[64\] = \{(.*?)\};", text, re.S).group(1)
    vals = [int(v) for v in re.findall(r"-?\d+", body)]
    assert len(vals) == 64 * 64
    return np.array(vals, dtype=np.int64).reshape(64, 64)


def table(n):
    """N-point integer DCT-2 as the kernels index it: row k of the 64-point
    table taken every 64 / N rows, first N columns."""
    return c2_64()[:: 64 // n, :n]


def extremes(t, sc, s):
    """Largest and smallest scaled sum and rounded result of t @ x over int16 x
    (each row taken at its worst inputs), with the offset 2^(s + sc - 1)."""
    tt = t * (1 << sc)
    hi = np.where(tt > 0, tt * XMAX, tt * XMIN).sum(axis=1).max() + (1 << (s + sc - 1))
    lo = np.where(tt > 0, tt * XMIN, tt * XMAX).sum(axis=1).min() + (1 << (s + sc - 1))
    return hi, lo, hi >> 16, lo >> 16


def test_table_is_the_nested_dct2():
    t = c2_64()
    assert (t[0] == 256).all()
    for n in (4, 8, 16, 32, 64):
        assert (np.abs(table(n)[n // 2]) == 256).all()          # row N/2: all +-2^8
    k = np.arange(64)[:, None]
    n = np.arange(64)[None, :]
    sym = np.where(k % 2 == 0, t[:, ::-1], -t[:, ::-1])       # T[k][N-1-n] = (-1)^k T[k][n]
    assert (t == sym).all()


@pytest.mark.parametrize("lh", [2, 3, 4, 5, 6])
def test_forward_column_stage_dct3_dst3(lh):
    """Forward column stage of a DCT-3 / DST-3 core: shift log2 H + 8, scale
    2^(8 - log2 H); the stage multiplies by the transposed table."""
    n = 1 << lh
    sc, s = 8 - lh, lh + 8
    t = table(n).T
    assert np.abs(t).sum(axis=1).max() < n * 256            # column L1 norm of the DCT-2 table
    assert np.abs(t).max() * (1 << sc) <= 32767              # scaled entries are int16 operands
    hi, lo, rhi, rlo = extremes(t, sc, s)
    assert hi < 2 ** 31 and lo >= -2 ** 31
    assert rhi <= XMAX and rlo >= XMIN


@pytest.mark.parametrize("lh", [2, 3, 4, 5, 6])
def test_forward_dct2_stage_is_not_scaled(lh):
    """A DCT-2 core (forward DCT-2, or a DCT-2 feeding a sub-block) cannot be
    scaled the same way: row N/2 of the table is all +-2^8, an L1 norm of
    N * 2^8 with mixed signs, so inputs of matching signs at +32767 / -32768
    push the scaled sum to 2^31 and the result past int16.  The packed
    kernels therefore keep the generic stage there."""
    n = 1 << lh
    hi, lo, rhi, rlo = extremes(table(n), 8 - lh, lh + 8)
    assert hi >= 2 ** 31 or rhi > XMAX


@pytest.mark.parametrize("lw", [2, 3, 4, 5])
@pytest.mark.parametrize("core", ["dct2", "dct3"])
def test_inverse_row_stage_at_bit_depth_8(lw, core):
    """Inverse row stage at bit depth 8 (shift 14, scale 4) for up to 32
    points, with either butterfly."""
    n = 1 << lw
    t = table(n) if core == "dct2" else table(n).T
    assert np.abs(t).max() * 4 <= 32767
    hi, lo, rhi, rlo = extremes(t, 2, 14)
    assert hi <= 2 ** 30 + 2 ** 15 and lo >= -2 ** 30
    assert rhi <= 2 ** 14 and rlo >= -2 ** 14


def test_inverse_row_stage_is_not_scaled_at_64_points():
    """At 64 points the DCT-2 rows would overflow int32 with scale 4, which is
    why the packed kernels keep the generic path there."""
    hi, lo, _, _ = extremes(table(64), 2, 14)
    assert lo < -2 ** 31 or hi >= 2 ** 31
