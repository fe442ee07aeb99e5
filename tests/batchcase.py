"""Batched uneven-block workload helpers (test side): frame partitions from
``synth``, block descriptors for the library, and the oracle's expected frames."""

import numpy as np

from oracle import fixed as F
from oracle import fp as P
from tests.cfgs import type_axis

from paper_2505_23618_amd.frames import SIZES, axis_id, descriptors, register_axes  # noqa: F401


def oracle_frames(frames, rows, params, inverse=False, select=None, bd=8):
    """Expected output frames (forward or inverse) for the blocks in `rows`
    (or only the indices in `select`), computed by the oracle per group of
    equal (w, h, type_h, type_v), at bit depth `bd`."""
    out = np.zeros_like(frames, dtype=np.int64)
    sel = np.arange(len(rows)) if select is None else np.asarray(select)
    keys = {}
    for i in sel:
        f, x, y, w, h, th, tv = (int(v) for v in rows[i])
        keys.setdefault((w, h, th, tv), []).append(i)
    for (w, h, th, tv), idx in keys.items():
        stack = np.stack([frames[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] for i in idx])
        ah, av = type_axis(params, th, w), type_axis(params, tv, h)
        res = F.inv2d(stack, ah, av, bd=bd) if inverse else F.fwd2d(stack, ah, av, bd=bd)
        for j, i in enumerate(idx):
            out[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] = res[j]
    return out


def oracle_frames_fp(frames, rows, params, inverse=False, select=None):
    """Expected fp64 output frames of the orthonormal transforms (the fp32
    path's reference) for the blocks in `rows` (or the indices in `select`)."""
    out = np.zeros(frames.shape, dtype=np.float64)
    sel = np.arange(len(rows)) if select is None else np.asarray(select)
    keys = {}
    for i in sel:
        f, x, y, w, h, th, tv = (int(v) for v in rows[i])
        keys.setdefault((w, h, th, tv), []).append(i)
    for (w, h, th, tv), idx in keys.items():
        stack = np.stack([frames[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w]
                          for i in idx]).astype(np.float64)
        ah, av = type_axis(params, th, w), type_axis(params, tv, h)
        res = P.inv2d(stack, ah, av) if inverse else P.fwd2d(stack, ah, av)
        for j, i in enumerate(idx):
            out[rows[i, 0], rows[i, 2]:rows[i, 2] + h, rows[i, 1]:rows[i, 1] + w] = res[j]
    return out


def block_rel_errors(got, ref, rows, select=None):
    """Per block: max |got - ref| / max |ref| (0 / 0 counts as 0, x / 0 as inf)."""
    sel = np.arange(len(rows)) if select is None else np.asarray(select)
    errs = np.empty(len(sel))
    for k, i in enumerate(sel):
        f, x, y, w, h = (int(v) for v in rows[i, :5])
        g = got[f, y:y + h, x:x + w].astype(np.float64)
        r = ref[f, y:y + h, x:x + w]
        e, sc = np.abs(g - r).max(), np.abs(r).max()
        errs[k] = 0.0 if e == 0 else (e / sc if sc > 0 else np.inf)
    return errs
