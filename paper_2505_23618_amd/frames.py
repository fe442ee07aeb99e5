"""Block-list helpers for frame workloads (host-side marshalling only).

Turns a frame partition (rows of (frame, x, y, w, h, type_h, type_v)) into
``ta_block`` descriptors for ``Plan``, and registers one library axis per
(transform type, block size): type 0 = DCT-2, 1 = adjusted DST-7 (DST-3 +
4-tap band fitted for that size), 2 = adjusted DCT-8 (the same band, flipped).
"""

from __future__ import annotations

import numpy as np

from . import ADJ_BAND, BLOCK_DTYPE, DCT2, DST3

SIZES = (4, 8, 16, 32, 64)


def axis_id(t: int, n: int) -> int:
    return 64 + 8 * t + int(np.log2(n))


def register_axes(ctx, ids: dict) -> None:
    for n in SIZES:
        ctx.axis(axis_id(0, n), DCT2)
        for t in (1, 2):
            ctx.axis(axis_id(t, n), DST3, ADJ_BAND, t == 2, ids[f"band_S3_S7_N{n}_K4"])


def descriptors(rows: np.ndarray, frame_h: int, frame_w: int) -> np.ndarray:
    """Same-geometry input and output frames: offset frame*H*W + y*W + x."""
    d = np.zeros(len(rows), BLOCK_DTYPE)
    off = rows[:, 0].astype(np.int64) * frame_h * frame_w + rows[:, 2].astype(np.int64) * frame_w + rows[:, 1]
    d["in_off"] = off
    d["out_off"] = off
    d["in_stride"] = frame_w
    d["out_stride"] = frame_w
    d["log2w"] = np.log2(rows[:, 3]).astype(np.uint8)
    d["log2h"] = np.log2(rows[:, 4]).astype(np.uint8)
    d["axis_h"] = [axis_id(int(t), int(n)) for t, n in zip(rows[:, 5], rows[:, 3])]
    d["axis_v"] = [axis_id(int(t), int(n)) for t, n in zip(rows[:, 6], rows[:, 4])]
    return d
