"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""

import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

import paper_2505_23618_amd as ta

HEADER = Path(__file__).resolve().parent.parent / "include" / "tadj.h"


def declared_symbols():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ta_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ta.lib()
    syms = declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(lib, s), s
    assert set(ta.EXPORTS) <= set(syms)


def test_version_string():
    assert b"gfx950" in ta.lib().ta_version()


def test_create_rejects_bad_arguments_without_gpu():
    lib = ta.lib()
    h = ctypes.c_void_p()
    assert lib.ta_create(None, 0, 8, 8, 10) == ta.TA_EINVAL
    for m in (5, 10):
        assert lib.ta_create(ctypes.byref(h), 0, 8, m, 10) == ta.TA_EUNSUPPORTED
        assert b"precision" in lib.ta_last_error()
    assert lib.ta_create(ctypes.byref(h), 0, 7, 6, 10) == ta.TA_EUNSUPPORTED   # bd + m < 14
    assert b"shift" in lib.ta_last_error()
    assert lib.ta_create(ctypes.byref(h), 0, 30, 8, 10) == ta.TA_EUNSUPPORTED
    assert lib.ta_create(ctypes.byref(h), 0, 8, 8, 20) == ta.TA_EUNSUPPORTED


def test_null_context_paths():
    lib = ta.lib()
    a = np.zeros((8, 8), np.int16)
    f = np.zeros((8, 8), np.float32)
    assert lib.ta_destroy(None) == ta.TA_EINVAL
    assert lib.ta_set_band(None, 0, 8, 4, a.ctypes.data, f.ctypes.data) == ta.TA_EINVAL
    assert lib.ta_set_post(None, 0, 8, 4, a.ctypes.data, f.ctypes.data) == ta.TA_EINVAL
    assert lib.ta_set_axis(None, 0, None) == ta.TA_EINVAL
    assert lib.ta_fwd_packed(None, 0, 0, 5, 5, 1, None, None, 0, None) == ta.TA_EINVAL
    assert lib.ta_inv_packed(None, 0, 0, 5, 5, 1, None, None, 0, None) == ta.TA_EINVAL
    assert lib.ta_set_impl(None, 0) == ta.TA_EINVAL
    assert lib.ta_fwd_multi(None, 0, 5, 1, None, None, None) == ta.TA_EINVAL


def test_coef_stats_argument_checks_without_gpu():
    lib = ta.lib()
    assert lib.ta_coef_stats(None, None, 1, 5, 5, 8, 4, None, None, None, None, None, None, None, 0,
                             None) == ta.TA_EINVAL
    assert lib.ta_coef_stats_workspace(None, 1, 5, 5, None) == ta.TA_EINVAL
    b = ctypes.c_int64(0)
    assert lib.ta_coef_stats_workspace(None, 1, 5, 5, ctypes.byref(b)) == ta.TA_EINVAL


def test_design_search_argument_checks_without_gpu():
    lib = ta.lib()
    assert lib.ta_design_search(None, 8, 1, None, 1, None, None, 1, 0.01, 1.0, None, None, None,
                                None) == ta.TA_EINVAL


def test_block_list_entry_points_reject_bad_arguments_without_gpu():
    lib = ta.lib()
    bad = ctypes.c_int64(7)
    assert lib.ta_transform_fwd(None, None, 1, None, None, ta.I16, None) == ta.TA_EINVAL
    assert lib.ta_transform_inv(None, None, 1, None, None, ta.I16, None) == ta.TA_EINVAL
    assert lib.ta_validate_blocks(None, None, 1, 0, 0, ctypes.byref(bad)) == ta.TA_EINVAL
    assert lib.ta_set_axis_cfg(None, 0, None) == ta.TA_EINVAL
    assert lib.ta_plan_tuning(None, None, None) == ta.TA_EINVAL
    assert lib.ta_plan_set_tuning(None, 1024, 20) == ta.TA_EINVAL
    nb = ctypes.c_int(0)
    assert lib.ta_plan_tile_blocks(None, 3, 3, ctypes.byref(nb)) == ta.TA_EINVAL
    assert lib.ta_plan_set_tile_blocks(None, 3, 3, 1) == ta.TA_EINVAL
    assert lib.ta_transform_fwd_ws(None, None, 1, None, None, ta.I16, None, 0, None) == ta.TA_EINVAL
    assert lib.ta_transform_inv_ws(None, None, 1, None, None, ta.I16, None, 0, None) == ta.TA_EINVAL
    ws = ctypes.c_int64(-1)
    assert lib.ta_transform_workspace(-1, ctypes.byref(ws)) == ta.TA_EINVAL
    assert lib.ta_transform_workspace(5, None) == ta.TA_EINVAL
    assert lib.ta_transform_workspace(0, ctypes.byref(ws)) == ta.TA_OK and ws.value == 0
    sizes = []
    for n in (1, 4096, 4097, 582094):
        assert lib.ta_transform_workspace(n, ctypes.byref(ws)) == ta.TA_OK
        sizes.append(ws.value)
    # 8 bytes of per-block data and at least one 80-byte tile slot per block
    assert all(s >= 88 * n for s, n in zip(sizes, (1, 4096, 4097, 582094))) and sizes == sorted(sizes)
    lay = np.array([ta.ADJ_BAND, 8, 4], np.int32)
    a = np.zeros(64, np.int16)
    f = np.zeros(64, np.float32)
    assert lib.ta_set_params(None, 0, a.ctypes.data, f.ctypes.data, lay.ctypes.data, 64) == ta.TA_EINVAL


def test_axis_cfg_struct_layout():
    assert ctypes.sizeof(ta._AxisCfg) == 24
    assert ctypes.sizeof(ta._Axis) == 16
