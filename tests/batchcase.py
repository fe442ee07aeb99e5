"""Batched uneven-block workload helpers (test side): frame partitions from
``synth``, block descriptors for the library, and the oracle's expected frames."""

import numpy as np

import paper_2505_23618_amd as ta
import synth
from oracle import fixed as F
from tests.cfgs import type_axis

SIZES = (4, 8, 16, 32, 64)


def axis_id(t, n):
    return 64 + 8 * t + int(np.log2(n))


def register_axes(ctx, ids):
    """One library axis per (type, size): 0 DCT-2, 1 adjusted DST-7, 2 adjusted DCT-8."""
    for n in SIZES:
        ctx.axis(axis_id(0, n), ta.DCT2)
        for t in (1, 2):
            ctx.axis(axis_id(t, n), ta.DST3, ta.ADJ_BAND, t == 2, ids[f"band_S3_S7_N{n}_K4"])


def descriptors(rows, frame_h, frame_w):
    """rows: int32 [n, 7] (frame, x, y, w, h, type_h, type_v) -> BLOCK_DTYPE."""
    d = np.zeros(len(rows), ta.BLOCK_DTYPE)
    off = rows[:, 0].astype(np.int64) * frame_h * frame_w + rows[:, 2].astype(np.int64) * frame_w + rows[:, 1]
    d["in_off"] = off
    d["out_off"] = off
    d["in_stride"] = frame_w
    d["out_stride"] = frame_w
    d["log2w"] = np.log2(rows[:, 3]).astype(np.uint8)
    d["log2h"] = np.log2(rows[:, 4]).astype(np.uint8)
    d["axis_h"] = [axis_id(t, n) for t, n in zip(rows[:, 5], rows[:, 3])]
    d["axis_v"] = [axis_id(t, n) for t, n in zip(rows[:, 6], rows[:, 4])]
    return d


def oracle_frames(frames, rows, params, inverse=False, select=None):
    """Expected output frames (forward or inverse) for the blocks in `rows`
    (or only the indices in `select`), computed by the oracle per group of
    equal (w, h, type_h, type_v)."""
    out = np.zeros_like(frames, dtype=np.int64)
    sel = np.arange(len(rows)) if select is None else np.asarray(select)
    keys = {}
    for i in sel:
        f, x, y, w, h, th, tv = (int(v) for v in rows[i])
        keys.setdefault((w, h, th, tv), []).append(i)
    for (w, h, th, tv), idx in keys.items():
        stack = np.stack([frames[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] for i in idx])
        ah, av = type_axis(params, th, w), type_axis(params, tv, h)
        res = F.inv2d(stack, ah, av) if inverse else F.fwd2d(stack, ah, av)
        for j, i in enumerate(idx):
            out[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] = res[j]
    return out
