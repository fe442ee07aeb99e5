"""The library's integer base tables (ta_int_table, host code, no GPU) at
every precision m in 6..9: equal to the oracle's tables (round half away of
2^m sqrt(N) times the orthonormal matrix, DCT-3 / DST-2 / DST-3 from the
DCT-2 by the section 2.1 relations), and at m = 8 equal to the tables
compiled into the specialised kernels (csrc/tables_gen.h, the nested 64-point
DCT-2 and the DST-7 tables), so contexts at m = 8 and at other m apply one
definition."""

import re
from pathlib import Path

import numpy as np
import pytest

import paper_2505_23618_amd as ta
from oracle import fixed as F

NAMES = {ta.DCT2: "C2", ta.DCT3: "C3", ta.DST2: "S2", ta.DST3: "S3", ta.DST7: "S7", ta.DCT8: "C8"}
TABLES = Path(__file__).resolve().parent.parent / "paper_2505_23618_amd" / "csrc" / "tables_gen.h"


@pytest.mark.parametrize("m", [6, 7, 8, 9])
@pytest.mark.parametrize("kind", list(NAMES))
def test_library_tables_equal_oracle(kind, m):
    for n in (4, 8, 16, 32, 64):
        assert (ta.int_table(kind, n, m) == F.int_table(NAMES[kind], n, m)).all(), (NAMES[kind], n, m)


def _compiled(name, n):
    body = re.search(rf"{name}\[{n}\]\[{n}\] = \{{(.*?)\}};", TABLES.read_text(), re.S).group(1)
    return np.array([int(v) for v in re.findall(r"-?\d+", body)], dtype=np.int64).reshape(n, n)


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_m8_tables_equal_compiled_tables(n):
    c2 = _compiled("ta_c2_64", 64)[:: 64 // n, :n]
    assert (ta.int_table(ta.DCT2, n, 8) == c2).all()
    assert (ta.int_table(ta.DST7, n, 8) == _compiled(f"ta_s7_{n}", n)).all()


def test_int_table_rejects_bad_arguments():
    out = np.zeros((8, 8), np.int16)
    lib = ta.lib()
    assert lib.ta_int_table(7, 8, 8, out.ctypes.data) == ta.TA_EINVAL
    assert lib.ta_int_table(ta.DCT2, 12, 8, out.ctypes.data) == ta.TA_EUNSUPPORTED
    assert lib.ta_int_table(ta.DCT2, 8, 10, out.ctypes.data) == ta.TA_EUNSUPPORTED
    assert lib.ta_int_table(ta.DCT2, 8, 8, None) == ta.TA_EINVAL
