"""The adjustment design study of section 2 (Fig. 1) on the GPU.

Fig. 1 shows, for each efficient base B in {DCT-2, DCT-3, DST-2, DST-3} and
each desired transform D among the other DSTs, the adjustment that minimises
the printed sparsity objective, with either A or C the identity.  This module
builds those candidate sets (the transform matrices, and per candidate the
base, target, pre/post mode and the sign sigma that makes the exact
adjustment reachable by M = G(theta) J) and runs them through
``ta_design_search``: every objective, gradient and Adam step runs in the HIP
kernel; the host only prepares the matrices and reads the results back.

Matrix orientation: rows are basis vectors (k = frequency), forward y = T x.
The DST-7 is the one of the codec (section 2.1); DST-6 is its transpose.
"""

from __future__ import annotations

import numpy as np

BASES = ("C2", "C3", "S2", "S3")
TARGETS = ("S1", "S4", "S5", "S6", "S7", "S8")
MODES = ("pre", "post")


def transform_matrix(kind: str, n: int) -> np.ndarray:
    """Orthonormal N-point trigonometric transform matrices, FP64."""
    k = np.arange(n, dtype=np.float64)[:, None]
    x = np.arange(n, dtype=np.float64)[None, :]
    pi = np.pi
    if kind == "C2":
        t = np.cos(pi * k * (2 * x + 1) / (2 * n)) * np.sqrt(2.0 / n)
        t[0] /= np.sqrt(2.0)
        return t
    if kind == "C3":
        return transform_matrix("C2", n).T.copy()
    if kind == "S2":
        t = np.sin(pi * (k + 1) * (2 * x + 1) / (2 * n)) * np.sqrt(2.0 / n)
        t[n - 1] /= np.sqrt(2.0)
        return t
    if kind == "S3":
        return transform_matrix("S2", n).T.copy()
    if kind == "S1":
        return np.sin(pi * (k + 1) * (x + 1) / (n + 1)) * np.sqrt(2.0 / (n + 1))
    if kind == "S4":
        return np.sin(pi * (2 * k + 1) * (2 * x + 1) / (4 * n)) * np.sqrt(2.0 / n)
    if kind == "S5":
        return np.sin(2 * pi * (k + 1) * (x + 1) / (2 * n + 1)) * (2.0 / np.sqrt(2 * n + 1))
    if kind == "S6":
        return transform_matrix("S7", n).T.copy()
    if kind == "S7":
        return np.sin(pi * (2 * k + 1) * (x + 1) / (2 * n + 1)) * np.sqrt(4.0 / (2 * n + 1))
    if kind == "S8":
        t = np.sin(pi * (2 * k + 1) * (2 * x + 1) / (4 * n - 2)) * np.sqrt(4.0 / (2 * n - 1))
        t[n - 1] /= np.sqrt(2.0)
        t[:, n - 1] /= np.sqrt(2.0)
        return t
    raise ValueError(kind)


def n_angles(n: int) -> int:
    return n * (n - 1) // 2


def study(n: int, restarts: int):
    """Matrices [nmat, n, n] (BASES then TARGETS), candidate rows
    [ncand, 4] int32 (base, target, mode, sigma) and their labels, for every
    (target, base, mode) and `restarts` starts each."""
    names = BASES + TARGETS
    mats = np.stack([transform_matrix(k, n) for k in names])
    rows, labels = [], []
    for ti, tk in enumerate(TARGETS):
        d = mats[len(BASES) + ti]
        for bi, bk in enumerate(BASES):
            b = mats[bi]
            for mi, mode in enumerate(MODES):
                tgt = b.T @ d if mode == "pre" else d @ b.T
                sigma = 1 if np.linalg.det(tgt) > 0 else -1
                for _ in range(restarts):
                    rows.append((bi, len(BASES) + ti, mi, sigma))
                    labels.append((bk, tk, mode))
    return mats, np.array(rows, dtype=np.int32), labels


def algorithmic_flops(n: int) -> float:
    """FP64 operations of one objective-and-gradient evaluation plus one Adam
    update: rotations forward (6 per angle and column) and backward (12 for
    the two transposed rotations, 3 for the angle-gradient term), the two
    N^3 products, the elementwise terms, and Adam (about 12 per angle)."""
    na = n_angles(n)
    return na * n * (6 + 15) + 4.0 * n ** 3 + 16.0 * n * n + 12.0 * na


def run_study(ctx, n: int, restarts: int, steps: int, lr: float, lam: float, starts: np.ndarray,
              sparse_threshold: float = 0.1):
    """Runs the whole study in one launch; per (target, base, mode) keeps the
    restart with the lowest objective.  Returns (rows, table) where table is a
    list of dicts (target, base, mode, objective, sparsity, error, nonzeros)."""
    import torch
    mats, cands, labels = study(n, restarts)
    dev = torch.device("cuda", ctx.device)
    m = torch.from_numpy(mats).to(dev)
    c = torch.from_numpy(cands).to(dev)
    th = torch.from_numpy(np.ascontiguousarray(starts, dtype=np.float64)).to(dev)
    out = ctx.design_search(m, c, th, steps, lr, lam, want_adj=True)
    obj = out["obj"].cpu().numpy()
    adj = out["adj"].cpu().numpy()
    best = {}
    for i, key in enumerate(labels):
        if key not in best or obj[i, 0] < obj[best[key], 0]:
            best[key] = i
    table = []
    for key, i in best.items():
        table.append({"base": key[0], "target": key[1], "mode": key[2], "objective": float(obj[i, 0]),
                      "sparsity": float(obj[i, 1]), "error": float(obj[i, 2]),
                      "nonzeros": int((np.abs(adj[i]) > sparse_threshold).sum())})
    return cands, table
