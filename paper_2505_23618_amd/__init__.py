"""Python binding of libtadj (batched 2-D adjusted DCT/DST transforms, gfx950).

A thin ctypes layer over the C ABI in include/tadj.h: it marshals torch
tensors (device memory) and the current HIP stream into the library calls.
All transform arithmetic runs in the library's HIP kernels; if the library
has not been built this module raises instead of falling back to anything.

    import paper_2505_23618_amd as ta
    ctx = ta.Context(device=0)
    ids = ta.load_params(ctx)                      # frozen adjustment parameters
    ax = ctx.axis(1, base=ta.DST3, adj=ta.ADJ_BAND, param=ids["band_S3_S7_N32_K4"])
    y = ctx.fwd(x_int16_cuda, ax, ax)              # x: [nblocks, H, W]
    x2 = ctx.inv(y, ax, ax)
"""

from __future__ import annotations

import ctypes
import json
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libtadj.so"
PARAMS_PATH = _PKG / "params" / "adjust_params.json"

# enums of tadj.h
I16, F32 = 0, 1
DCT2, DCT3, DST2, DST3, DST7, DCT8 = range(6)
ADJ_NONE, ADJ_BAND, ADJ_POST = range(3)
BASES = {"C2": DCT2, "C3": DCT3, "S2": DST2, "S3": DST3, "S7": DST7, "C8": DCT8}

TA_OK, TA_EINVAL, TA_EUNSUPPORTED, TA_ENOPARAMS, TA_EHIP = 0, -1, -2, -3, -4

EXPORTS = ("ta_create", "ta_destroy", "ta_set_band", "ta_set_post", "ta_set_axis",
           "ta_fwd_packed", "ta_inv_packed", "ta_set_impl", "ta_version", "ta_last_error",
           "ta_plan_create", "ta_plan_destroy", "ta_plan_info", "ta_plan_fwd", "ta_plan_inv",
           "ta_plan_autotune", "ta_givens_workspace", "ta_givens_fwd", "ta_givens_bwd",
           "ta_fwd_multi", "ta_coef_stats_workspace", "ta_coef_stats", "ta_design_search",
           "ta_transform_fwd", "ta_transform_inv", "ta_validate_blocks", "ta_set_axis_cfg", "ta_set_params",
           "ta_plan_tuning", "ta_plan_set_tuning", "ta_plan_extents", "ta_givens_bwd_noalloc",
           "ta_int_table", "ta_set_band_angles", "ta_set_post_angles", "ta_transform_bwd",
           "ta_plan_tile_blocks", "ta_plan_set_tile_blocks", "ta_transform_workspace", "ta_transform_fwd_ws",
           "ta_transform_inv_ws")

# ta_block (32 bytes), as a numpy structured dtype
BLOCK_DTYPE = np.dtype([("in_off", "<i8"), ("out_off", "<i8"), ("in_stride", "<i4"), ("out_stride", "<i4"),
                        ("log2w", "u1"), ("log2h", "u1"), ("axis_h", "<u2"), ("axis_v", "<u2"),
                        ("reserved", "<u2")])
assert BLOCK_DTYPE.itemsize == 32


class TadjError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tadj error {code}: {msg}")
        self.code = code


class _Axis(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int32), ("adj", ctypes.c_int32),
                ("flip", ctypes.c_int32), ("param_id", ctypes.c_int32)]


class _AxisCfg(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int32), ("adj", ctypes.c_int32), ("flip", ctypes.c_int32),
                ("log2n", ctypes.c_int32), ("k_or_b", ctypes.c_int32), ("param_id", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libtadj.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_23618_amd.build`")
    L = ctypes.CDLL(str(LIB_PATH))
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    L.ta_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32]
    L.ta_destroy.argtypes = [vp]
    L.ta_set_band.argtypes = [vp, i32, i32, i32, vp, vp]
    L.ta_set_post.argtypes = [vp, i32, i32, i32, vp, vp]
    L.ta_set_axis.argtypes = [vp, i32, ctypes.POINTER(_Axis)]
    for f in (L.ta_fwd_packed, L.ta_inv_packed):
        f.argtypes = [vp, i32, i32, i32, i32, i64, vp, vp, i32, vp]
    L.ta_set_impl.argtypes = [vp, i32]
    L.ta_fwd_multi.argtypes = [vp, i32, i32, i64, vp, vp, vp]
    L.ta_design_search.argtypes = [vp, i32, i32, vp, i64, vp, vp, i32, ctypes.c_double, ctypes.c_double,
                                   vp, vp, vp, vp]
    L.ta_coef_stats_workspace.argtypes = [vp, i64, i32, i32, ctypes.POINTER(i64)]
    L.ta_coef_stats.argtypes = [vp, vp, i64, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    L.ta_plan_create.argtypes = [vp, vp, i64, i32, ctypes.POINTER(vp)]
    L.ta_plan_destroy.argtypes = [vp]
    L.ta_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.ta_plan_fwd.argtypes = [vp, vp, vp, vp, vp]
    L.ta_plan_inv.argtypes = [vp, vp, vp, vp, vp]
    L.ta_plan_autotune.argtypes = [vp, vp, vp, vp, vp, i32]
    L.ta_plan_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.ta_plan_set_tuning.argtypes = [vp, i32, i32]
    L.ta_plan_tile_blocks.argtypes = [vp, i32, i32, ctypes.POINTER(i32)]
    L.ta_plan_set_tile_blocks.argtypes = [vp, i32, i32, i32]
    L.ta_plan_extents.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.ta_givens_workspace.argtypes = [i64, ctypes.POINTER(i64)]
    L.ta_givens_fwd.argtypes = [vp, i32, i32, i32, vp, i64, vp, vp, vp]
    L.ta_givens_bwd.argtypes = [vp, i32, i32, i32, vp, i64, vp, vp, vp, vp, vp, vp]
    L.ta_givens_bwd_noalloc.argtypes = [vp, i32, i32, i32, vp, i64, vp, vp, vp, vp, vp]
    L.ta_int_table.argtypes = [i32, i32, i32, vp]
    L.ta_set_band_angles.argtypes = [vp, i32, i32, i32, vp]
    L.ta_set_post_angles.argtypes = [vp, i32, i32, i32, vp, vp]
    L.ta_transform_bwd.argtypes = [vp, vp, i64, vp, vp, vp, vp, i32, vp]
    for f in (L.ta_transform_fwd, L.ta_transform_inv):
        f.argtypes = [vp, vp, i64, vp, vp, i32, vp]
    for f in (L.ta_transform_fwd_ws, L.ta_transform_inv_ws):
        f.argtypes = [vp, vp, i64, vp, vp, i32, vp, i64, vp]
    L.ta_transform_workspace.argtypes = [i64, ctypes.POINTER(i64)]
    L.ta_validate_blocks.argtypes = [vp, vp, i64, i64, i64, ctypes.POINTER(i64)]
    L.ta_set_axis_cfg.argtypes = [vp, i32, ctypes.POINTER(_AxisCfg)]
    L.ta_set_params.argtypes = [vp, i32, vp, vp, vp, i64]
    L.ta_version.restype = ctypes.c_char_p
    L.ta_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("ta_version", "ta_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


SUMMARY_FIELDS = ("bits_per_coef", "mse_per_coef", "energy_per_coef", "coding_gain_db",
                  "low_band_fraction", "nonzero_fraction", "escape_fraction")
STATS_SYMBOLS = 65      # levels -31..31 and the two escapes


def _check(code: int):
    if code != 0:
        raise TadjError(code, lib().ta_last_error().decode())


def _check_side(n: int):
    if n < 4 or n > 64 or n & (n - 1):
        raise ValueError(f"block side {n}: sides are powers of two in 4..64")


def _check_out(out, shape, dtype, device):
    """A caller-supplied output must be exactly what the kernel writes: the
    C ABI receives only its pointer, so a smaller or differently typed tensor
    would be written past its end."""
    if tuple(out.shape) != tuple(shape) or out.dtype != dtype or out.device != device:
        raise ValueError(f"out must be {dtype} {tuple(shape)} on {device}, got {out.dtype} "
                         f"{tuple(out.shape)} on {out.device}")
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A libtadj context on one GPU (owns the device parameter tables)."""

    def __init__(self, device: int = 0, bit_depth: int = 8, m: int = 8, a: int = 10):
        self._h = ctypes.c_void_p()
        _check(lib().ta_create(ctypes.byref(self._h), device, bit_depth, m, a))
        self.device, self.bit_depth, self.m, self.a = device, bit_depth, m, a

    def close(self):
        if self._h:
            lib().ta_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration --------------------------------------------------------
    def set_band(self, pid: int, a_int: np.ndarray, a_f32: np.ndarray, taps: int):
        a_int = np.ascontiguousarray(a_int, dtype=np.int16)
        a_f32 = np.ascontiguousarray(a_f32, dtype=np.float32)
        n = a_int.shape[0]
        _check(lib().ta_set_band(self._h, pid, n, taps, a_int.ctypes.data, a_f32.ctypes.data))

    def set_post(self, pid: int, q_int: np.ndarray, q_f32: np.ndarray, n: int):
        q_int = np.ascontiguousarray(q_int, dtype=np.int16)
        q_f32 = np.ascontiguousarray(q_f32, dtype=np.float32)
        _check(lib().ta_set_post(self._h, pid, n, q_int.shape[0], q_int.ctypes.data, q_f32.ctypes.data))

    def axis(self, aid: int, base: int, adj: int = ADJ_NONE, flip: bool = False, param: int = 0) -> int:
        ax = _Axis(base, adj, int(bool(flip)), param)
        _check(lib().ta_set_axis(self._h, aid, ctypes.byref(ax)))
        return aid

    def axis_cfg(self, aid: int, base: int, adj: int = ADJ_NONE, flip: bool = False, log2n: int = 0,
                 k_or_b: int = 0, param: int = 0) -> int:
        """ta_set_axis_cfg: as axis(), with the size and K/B stated (checked against the set)."""
        cfg = _AxisCfg(base, adj, int(bool(flip)), log2n, k_or_b, param)
        _check(lib().ta_set_axis_cfg(self._h, aid, ctypes.byref(cfg)))
        return aid

    def set_params(self, pid: int, layout, int_taps: np.ndarray, f32_params: np.ndarray):
        """ta_set_params with layout = (adj, size, k_or_b)."""
        int_taps = np.ascontiguousarray(int_taps, dtype=np.int16).ravel()
        f32_params = np.ascontiguousarray(f32_params, dtype=np.float32).ravel()
        if int_taps.size != f32_params.size:
            raise ValueError("int_taps and f32_params differ in size")
        lay = np.ascontiguousarray(layout, dtype=np.int32)
        if lay.shape != (3,):
            raise ValueError("layout is (adj, size, k_or_b)")
        _check(lib().ta_set_params(self._h, pid, int_taps.ctypes.data, f32_params.ctypes.data, lay.ctypes.data,
                                   int_taps.size))

    def set_impl(self, impl: int):
        """0: matrix-core kernels for int16 transforms without a band adjustment
        where built, else VALU; 1: matrix cores only; 2: VALU only."""
        _check(lib().ta_set_impl(self._h, impl))

    # -- transforms -------------------------------------------------------------
    def _run(self, fn, x, axis_h, axis_v, out):
        import torch
        if x.dim() != 3:
            raise ValueError("expected [nblocks, H, W]")
        nb, h, w = x.shape
        _check_side(h)
        _check_side(w)
        lw, lh = w.bit_length() - 1, h.bit_length() - 1
        dt = {torch.int16: I16, torch.float32: F32}.get(x.dtype)
        if dt is None:
            raise TypeError(f"unsupported dtype {x.dtype}")
        if not x.is_cuda:
            raise ValueError("input must be a GPU tensor")
        x = x.contiguous()
        if out is None:
            out = torch.empty_like(x)
        else:
            _check_out(out, x.shape, x.dtype, x.device)
        _check(fn(self._h, axis_h, axis_v, lw, lh, nb, ctypes.c_void_p(x.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), dt, _stream_handle(None)))
        return out

    def fwd(self, x, axis_h: int, axis_v: int, out=None):
        """Forward 2-D transform of a packed batch [nblocks, H, W] (rows first)."""
        return self._run(lib().ta_fwd_packed, x, axis_h, axis_v, out)

    def inv(self, y, axis_h: int, axis_v: int, out=None):
        """Inverse 2-D transform of a packed batch (columns first)."""
        return self._run(lib().ta_inv_packed, y, axis_h, axis_v, out)

    def fwd_multi(self, x, param_id: int, out=None):
        """The five encoder transforms of a packed int16 batch [nblocks, N, N]
        (ta_fwd_multi): returns [5, nblocks, N, N] in the order DCT-2/DCT-2,
        (DST-7, DST-7), (DST-7, DCT-8), (DCT-8, DST-7), (DCT-8, DCT-8) as
        (vertical, horizontal)."""
        import torch
        if x.dim() != 3 or x.shape[1] != x.shape[2] or x.dtype != torch.int16 or not x.is_cuda:
            raise ValueError("expected a GPU int16 tensor [nblocks, N, N]")
        x = x.contiguous()
        nb, n = x.shape[0], x.shape[1]
        _check_side(n)
        if out is None:
            out = torch.empty((5, nb, n, n), dtype=torch.int16, device=x.device)
        else:
            _check_out(out, (5, nb, n, n), torch.int16, x.device)
        _check(lib().ta_fwd_multi(self._h, param_id, n.bit_length() - 1, nb, ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), _stream_handle(None)))
        return out

    def coef_stats(self, coef, step: int, offset: int, out=None):
        """Statistics of the quantised coefficients of a packed int16 batch
        [nblocks, H, W] (ta_coef_stats): a dict of GPU tensors hist [P, 65]
        (int32 view of the uint32 symbol counts, column 32 + symbol),
        esc_bits, energy, dist [P] (int64), rate [P] and summary [7]
        (float64; fields SUMMARY_FIELDS), P = H * W, plus the device scratch
        ("workspace").  `out`, a dict from an earlier call with the same
        block shape, is reused."""
        import torch
        if coef.dim() != 3 or coef.dtype != torch.int16 or not coef.is_cuda:
            raise ValueError("expected a GPU int16 tensor [nblocks, H, W]")
        coef = coef.contiguous()
        nb, h, w = coef.shape
        if h & (h - 1) or w & (w - 1) or h == 0 or w == 0:
            raise ValueError("block sides must be powers of two")
        p = h * w
        lh, lw = h.bit_length() - 1, w.bit_length() - 1
        ws = ctypes.c_int64(0)
        _check(lib().ta_coef_stats_workspace(self._h, nb, lh, lw, ctypes.byref(ws)))
        if out is None or out["workspace"].numel() < ws.value or out["hist"].shape[0] != p:
            dev = coef.device
            out = {"hist": torch.empty((p, STATS_SYMBOLS), dtype=torch.int32, device=dev),
                   "esc_bits": torch.empty(p, dtype=torch.int64, device=dev),
                   "energy": torch.empty(p, dtype=torch.int64, device=dev),
                   "dist": torch.empty(p, dtype=torch.int64, device=dev),
                   "rate": torch.empty(p, dtype=torch.float64, device=dev),
                   "summary": torch.empty(len(SUMMARY_FIELDS), dtype=torch.float64, device=dev),
                   "workspace": torch.empty(max(ws.value, 8), dtype=torch.uint8, device=dev)}
        ptr = {k: ctypes.c_void_p(v.data_ptr()) for k, v in out.items()}
        _check(lib().ta_coef_stats(self._h, ctypes.c_void_p(coef.data_ptr()), nb, lh, lw, step, offset,
                                   ptr["hist"], ptr["esc_bits"], ptr["energy"], ptr["dist"], ptr["rate"],
                                   ptr["summary"], ptr["workspace"], out["workspace"].numel(),
                                   _stream_handle(None)))
        return out

    def design_search(self, mats, cands, theta, steps: int, lr: float, lam: float = 1.0,
                      want_grad: bool = False, want_adj: bool = True):
        """Batched adjustment design search (ta_design_search) on GPU tensors:
        mats [nmat, n, n] float64, cands [ncand, 4] int32 (base, target,
        mode 0 pre / 1 post, sigma), theta [ncand, n(n-1)/2] float64 (start;
        overwritten with the result).  Returns a dict with obj [ncand, 3]
        (f, sparsity, error), and grad / adj when asked for."""
        import torch
        n = mats.shape[-1]
        ncand = cands.shape[0]
        if mats.dim() != 3 or mats.shape[1] != n or cands.dim() != 2 or cands.shape[1] != 4 or \
                tuple(theta.shape) != (ncand, n * (n - 1) // 2):
            raise ValueError("expected mats [nmat, n, n], cands [ncand, 4], theta [ncand, n(n-1)/2]")
        if mats.dtype != torch.float64 or theta.dtype != torch.float64 or cands.dtype != torch.int32:
            raise ValueError("mats and theta must be float64, cands int32")
        if not (mats.is_cuda and cands.is_cuda and theta.is_cuda):
            raise ValueError("expected GPU tensors")
        mats, cands = mats.contiguous(), cands.contiguous()
        if not theta.is_contiguous():
            raise ValueError("theta must be contiguous (it is overwritten)")
        dev = mats.device
        out = {"obj": torch.empty((ncand, 3), dtype=torch.float64, device=dev)}
        if want_grad:
            out["grad"] = torch.empty_like(theta)
        if want_adj:
            out["adj"] = torch.empty((ncand, n, n), dtype=torch.float64, device=dev)
        ptr = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None  # noqa: E731
        _check(lib().ta_design_search(self._h, n, mats.shape[0], ctypes.c_void_p(mats.data_ptr()), ncand,
                                      ctypes.c_void_p(cands.data_ptr()), ctypes.c_void_p(theta.data_ptr()), steps,
                                      lr, lam, ptr("grad"), ptr("obj"), ptr("adj"), _stream_handle(None)))
        return out

    # raw pointer variants (no allocation; for graphs and benchmarks)
    # -- unplanned block lists ----------------------------------------------------
    @staticmethod
    def blocks_to_device(blocks: np.ndarray, device: int = 0):
        """A ``BLOCK_DTYPE`` array as a uint8 [n, 32] tensor in device memory."""
        import torch
        blocks = np.ascontiguousarray(blocks, dtype=BLOCK_DTYPE)
        raw = torch.from_numpy(blocks.view(np.uint8).reshape(len(blocks), 32).copy())
        return raw.to(f"cuda:{device}")

    @staticmethod
    def _nblocks(blocks_dev) -> int:
        import torch
        if blocks_dev.dtype != torch.uint8 or blocks_dev.dim() != 2 or blocks_dev.shape[1] != 32:
            raise ValueError("descriptors are a uint8 [n, 32] device tensor (blocks_to_device)")
        if not blocks_dev.is_contiguous():
            raise ValueError("descriptors must be contiguous")
        return blocks_dev.shape[0]

    def _run_blocks(self, fn, blocks_dev, x, out, stream_handle):
        import torch
        n = self._nblocks(blocks_dev)
        if x.dtype != out.dtype or x.dtype not in (torch.int16, torch.float32):
            raise ValueError("block lists run on int16 (fixed point) or float32 buffers of one dtype")
        if not (x.is_contiguous() and out.is_contiguous()):
            raise ValueError("block lists need contiguous buffers")
        dt = I16 if x.dtype == torch.int16 else F32
        sh = _stream_handle(None) if stream_handle is None else ctypes.c_void_p(stream_handle)
        _check(fn(self._h, ctypes.c_void_p(blocks_dev.data_ptr()), n, ctypes.c_void_p(x.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), dt, sh))
        return out

    def transform_workspace(self, nblocks: int, device=None):
        """A uint8 device tensor of ta_transform_workspace(nblocks) bytes (256-byte aligned)."""
        import torch
        b = ctypes.c_int64(0)
        _check(lib().ta_transform_workspace(nblocks, ctypes.byref(b)))
        return torch.empty(max(b.value, 256), dtype=torch.uint8, device=f"cuda:{self.device}")

    def _run_blocks_ws(self, fn, blocks_dev, x, out, ws, stream_handle):
        import torch
        n = self._nblocks(blocks_dev)
        if x.dtype != out.dtype or x.dtype not in (torch.int16, torch.float32):
            raise ValueError("block lists run on int16 (fixed point) or float32 buffers of one dtype")
        if not (x.is_contiguous() and out.is_contiguous()):
            raise ValueError("block lists need contiguous buffers")
        if ws.dtype != torch.uint8 or not ws.is_contiguous():
            raise ValueError("the workspace is a contiguous uint8 device tensor (transform_workspace)")
        dt = I16 if x.dtype == torch.int16 else F32
        sh = _stream_handle(None) if stream_handle is None else ctypes.c_void_p(stream_handle)
        _check(fn(self._h, ctypes.c_void_p(blocks_dev.data_ptr()), n, ctypes.c_void_p(x.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), dt, ctypes.c_void_p(ws.data_ptr()), ws.numel(), sh))
        return out

    def transform_fwd_ws(self, blocks_dev, x, out, ws, stream_handle=None):
        """ta_transform_fwd_ws: the list planned on the device, then the planned kernel."""
        return self._run_blocks_ws(lib().ta_transform_fwd_ws, blocks_dev, x, out, ws, stream_handle)

    def transform_inv_ws(self, blocks_dev, y, out, ws, stream_handle=None):
        """ta_transform_inv_ws: the list planned on the device, then the planned kernel."""
        return self._run_blocks_ws(lib().ta_transform_inv_ws, blocks_dev, y, out, ws, stream_handle)

    def transform_fwd(self, blocks_dev, x, out, stream_handle=None):
        """ta_transform_fwd over descriptors already in device memory."""
        return self._run_blocks(lib().ta_transform_fwd, blocks_dev, x, out, stream_handle)

    def set_band_angles(self, pid: int, n: int, taps: int, theta):
        """ta_set_band_angles: band set `pid` as A(theta) (layers of Givens rotations)."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        _check(lib().ta_set_band_angles(self._h, pid, n, taps, th.ctypes.data))

    def set_post_angles(self, pid: int, n: int, b: int, phi, q0=None):
        """ta_set_post_angles: sub-block set `pid` as Q0 R(phi)."""
        ph = np.ascontiguousarray(phi, dtype=np.float64)
        q = None if q0 is None else np.ascontiguousarray(q0, dtype=np.float64)
        _check(lib().ta_set_post_angles(self._h, pid, n, b, None if q is None else q.ctypes.data, ph.ctypes.data))

    def transform_bwd(self, blocks_dev, x, gy, gx, gtheta, pid: int, stream_handle=None):
        """ta_transform_bwd over descriptors in device memory (fp32 buffers)."""
        import torch
        n = self._nblocks(blocks_dev)
        for t in (x, gy, gx, gtheta):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("the backward takes contiguous float32 GPU tensors")
        sh = _stream_handle(None) if stream_handle is None else ctypes.c_void_p(stream_handle)
        _check(lib().ta_transform_bwd(self._h, ctypes.c_void_p(blocks_dev.data_ptr()), n, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(gy.data_ptr()), ctypes.c_void_p(gx.data_ptr()),
                                      ctypes.c_void_p(gtheta.data_ptr()), pid, sh))
        return gx, gtheta

    def transform_inv(self, blocks_dev, y, out, stream_handle=None):
        """ta_transform_inv over descriptors already in device memory."""
        return self._run_blocks(lib().ta_transform_inv, blocks_dev, y, out, stream_handle)

    def validate_blocks(self, blocks_dev, in_elems: int, out_elems: int):
        """(-1, "") when every descriptor is valid, else (index of the first bad one, reason)."""
        n = self._nblocks(blocks_dev)
        bad = ctypes.c_int64(-1)
        code = lib().ta_validate_blocks(self._h, ctypes.c_void_p(blocks_dev.data_ptr()), n, in_elems, out_elems,
                                        ctypes.byref(bad))
        if code != 0 and bad.value < 0:
            _check(code)
        return bad.value, (lib().ta_last_error().decode() if code != 0 else "")

    def fwd_ptr(self, axis_h, axis_v, log2w, log2h, nblocks, in_ptr, out_ptr, dtype, stream_handle):
        _check(lib().ta_fwd_packed(self._h, axis_h, axis_v, log2w, log2h, nblocks,
                                   ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr), dtype,
                                   ctypes.c_void_p(stream_handle)))

    def inv_ptr(self, axis_h, axis_v, log2w, log2h, nblocks, in_ptr, out_ptr, dtype, stream_handle):
        _check(lib().ta_inv_packed(self._h, axis_h, axis_v, log2w, log2h, nblocks,
                                   ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr), dtype,
                                   ctypes.c_void_p(stream_handle)))


class Plan:
    """A batched plan over a list of uneven blocks (``BLOCK_DTYPE`` records)."""

    def __init__(self, ctx: Context, blocks: np.ndarray, dtype: int = I16):
        blocks = np.ascontiguousarray(blocks, dtype=BLOCK_DTYPE)
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        _check(lib().ta_plan_create(ctx._h, blocks.ctypes.data, len(blocks), dtype, ctypes.byref(self._h)))
        dt, ie, oe = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ta_plan_extents(self._h, ctypes.byref(dt), ctypes.byref(ie), ctypes.byref(oe)))
        self.dtype, self.in_elems, self.out_elems = dt.value, ie.value, oe.value

    def _check_buffers(self, x, out):
        """The kernels read and write every block the plan addresses: the
        buffers must hold them, in the plan's dtype, contiguous, on its GPU."""
        import torch
        want = torch.int16 if self.dtype == I16 else torch.float32
        for name, t, need in (("input", x, self.in_elems), ("output", out, self.out_elems)):
            if t.dtype != want:
                raise ValueError(f"{name} must be {want} for this plan, got {t.dtype}")
            if not t.is_cuda or t.device.index != self.ctx.device:
                raise ValueError(f"{name} must be on cuda:{self.ctx.device}")
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
            if t.numel() < need:
                raise ValueError(f"{name} holds {t.numel()} elements, the plan addresses {need}")
        if x.data_ptr() == out.data_ptr():
            raise ValueError("input and output must be different buffers")

    def close(self):
        if self._h:
            lib().ta_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        nb, nt, g, r = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        _check(lib().ta_plan_info(self._h, ctypes.byref(nb), ctypes.byref(nt), ctypes.byref(g)))
        _check(lib().ta_plan_tuning(self._h, ctypes.byref(g), ctypes.byref(r)))
        return {"blocks": nb.value, "tiles": nt.value, "grid": g.value, "region_log2": r.value}

    def fwd(self, x, out, stream_handle=None):
        self._check_buffers(x, out)
        sh = _stream_handle(None) if stream_handle is None else ctypes.c_void_p(stream_handle)
        _check(lib().ta_plan_fwd(self.ctx._h, self._h, ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), sh))
        return out

    def inv(self, y, out, stream_handle=None):
        self._check_buffers(y, out)
        sh = _stream_handle(None) if stream_handle is None else ctypes.c_void_p(stream_handle)
        _check(lib().ta_plan_inv(self.ctx._h, self._h, ctypes.c_void_p(y.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), sh))
        return out

    def set_tuning(self, grid: int, region_log2: int):
        _check(lib().ta_plan_set_tuning(self._h, grid, region_log2))
        return self.info()

    def tile_blocks(self):
        """Blocks per tile for each block size {(w, h): n} (the plan's choice)."""
        n = ctypes.c_int()
        res = {}
        for lw in range(2, 7):
            for lh in range(2, 7):
                _check(lib().ta_plan_tile_blocks(self._h, lw, lh, ctypes.byref(n)))
                res[(1 << lw, 1 << lh)] = n.value
        return res

    def set_tile_blocks(self, w: int, h: int, blocks: int):
        """Blocks per tile for w x h blocks (0: the kernels' maximum)."""
        _check_side(w)
        _check_side(h)
        _check(lib().ta_plan_set_tile_blocks(self._h, w.bit_length() - 1, h.bit_length() - 1, blocks))
        return self.info()

    def autotune(self, x, out, reps: int = 3):
        self._check_buffers(x, out)
        _check(lib().ta_plan_autotune(self.ctx._h, self._h, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _stream_handle(None), reps))
        return self.info()


def int_table(kind: int, n: int, m: int = 8) -> np.ndarray:
    """The library's integer base table (ta_int_table; no GPU needed)."""
    out = np.zeros((n, n), dtype=np.int16)
    _check(lib().ta_int_table(kind, n, m, out.ctypes.data))
    return out


def load_param_file(path: Path = PARAMS_PATH) -> dict:
    with open(path) as f:
        return {e["name"]: e for e in json.load(f)["entries"]}


def load_params(ctx: Context, path: Path = PARAMS_PATH) -> dict:
    """Register every frozen parameter set with the context; returns name -> id."""
    ids = {}
    for pid, (name, e) in enumerate(sorted(load_param_file(path).items())):
        if e["kind"] == "band":
            ctx.set_band(pid, np.asarray(e["a_int"]), np.asarray(e["a_f64"]), e["taps"])
        else:
            ctx.set_post(pid, np.asarray(e["q_int"]), np.asarray(e["q_f64"]), e["n"])
        ids[name] = pid
    return ids
