"""Seeded synthetic inputs for the adjusted-transform workloads.

This module is shared by the tests, the benchmark and the CPU oracle.  It only
draws random numbers and arranges them into residual blocks, residual vectors
and block partitions; it contains none of the transform arithmetic.

The paper measures inside a video codec on the JVET common-test-condition
sequences (section 3, Tables 2 and 3), which are not available here.  The
residuals are therefore synthesised from the first-order Gauss-Markov (AR(1))
model under which the DST-7 is the optimal transform for intra residuals
(introduction, the works cited for DST-7), and the frame partitions mimic a
quadtree/binary-tree split of 3840x2160 (class A) pictures.

AR(1) recipe (separable, innovation form, zero top/left boundary):
    X = L_H E L_W^T,  L[i, j] = rho**(i-j) for i >= j else 0,
    E iid N(0, sigma^2) (sigma is the innovation standard deviation),
then X is rounded to nearest (ties to even, ``numpy.rint``), clipped to
[-255, 255] and stored as int16.
"""

from __future__ import annotations

import hashlib

import numpy as np

SEED_BASE = 250523618


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ar1_filter(n: int, rho: float) -> np.ndarray:
    """Lower-triangular causal AR(1) synthesis filter L[i, j] = rho**(i-j)."""
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    lag = np.maximum(i - j, 0).astype(np.float64)
    return np.where(i >= j, rho ** lag, 0.0)


def ar1_blocks(nblocks: int, h: int, w: int, rho: float, sigma: float, seed: int,
               clip: int = 255, chunk: int = 16384) -> np.ndarray:
    """``nblocks`` H x W int16 residual blocks from the separable AR(1) model.

    Generated in chunks of ``chunk`` blocks so that the full 262,144-block
    workload never holds more than a few hundred MB of float64 at once; the
    random stream is consumed in block order, so the result does not depend on
    the chunk size.
    """
    rng = _rng(seed)
    lh = ar1_filter(h, rho)
    lw = ar1_filter(w, rho)
    out = np.empty((nblocks, h, w), dtype=np.int16)
    for s in range(0, nblocks, chunk):
        n = min(chunk, nblocks - s)
        e = rng.standard_normal((n, h, w)) * sigma
        t = (e.reshape(n * h, w) @ lw.T).reshape(n, h, w)          # rows: E L_W^T
        t = np.einsum("ij,bjk->bik", lh, t, optimize=True)        # cols: L_H (.)
        out[s:s + n] = np.clip(np.rint(t), -clip, clip).astype(np.int16)
    return out


def ar1_vectors(n: int, length: int, rho_lo: float, rho_hi: float, sigma: float,
                seed: int) -> np.ndarray:
    """``n`` float64 AR(1) vectors of ``length`` samples, rho ~ U[rho_lo, rho_hi]
    drawn per vector, innovation std ``sigma``, zero initial state."""
    rng = _rng(seed)
    rho = rng.uniform(rho_lo, rho_hi, size=n)
    e = rng.standard_normal((n, length)) * sigma
    x = np.empty((n, length), dtype=np.float64)
    x[:, 0] = e[:, 0]
    for t in range(1, length):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    return x


def adversarial_blocks(h: int, w: int, kind: str, seed: int = 0, n: int = 4) -> np.ndarray:
    """Edge-case int16 inputs: extreme residuals and full-range coefficients."""
    if kind == "zeros":
        return np.zeros((n, h, w), np.int16)
    if kind == "pos":
        return np.full((n, h, w), 255, np.int16)
    if kind == "neg":
        return np.full((n, h, w), -255, np.int16)
    if kind == "checker":
        r = np.arange(h)[:, None]
        c = np.arange(w)[None, :]
        b = np.where((r + c) % 2 == 0, 255, -255).astype(np.int16)
        return np.broadcast_to(b, (n, h, w)).copy()
    if kind == "uniform_res":
        return _rng(seed).integers(-255, 256, size=(n, h, w)).astype(np.int16)
    if kind == "full16":
        # full int16 range: what an inverse transform may be fed
        return _rng(seed).integers(-32768, 32768, size=(n, h, w)).astype(np.int16)
    if kind == "extreme16":
        v = _rng(seed).integers(0, 2, size=(n, h, w))
        return np.where(v == 0, -32768, 32767).astype(np.int16)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Frame partitions for the batched uneven workload
# --------------------------------------------------------------------------

# stop probability by the block's larger dimension; 4x4 always stops
_STOP = {64: 0.05, 32: 0.3, 16: 0.5, 8: 0.7}


def _split(rng, x, y, w, h, out):
    if w == 4 and h == 4:
        out.append((x, y, w, h))
        return
    big = max(w, h)
    if big <= 64 and rng.random() < _STOP.get(big, 0.7):
        out.append((x, y, w, h))
        return
    legal = []
    if w == h and w > 4:
        legal.append("qt")
    if h > 4:
        legal.append("bth")
    if w > 4:
        legal.append("btv")
    kind = legal[rng.integers(len(legal))]
    if kind == "qt":
        hw, hh = w // 2, h // 2
        for dy in (0, hh):
            for dx in (0, hw):
                _split(rng, x + dx, y + dy, hw, hh, out)
    elif kind == "bth":
        _split(rng, x, y, w, h // 2, out)
        _split(rng, x, y + h // 2, w, h // 2, out)
    else:
        _split(rng, x, y, w // 2, h, out)
        _split(rng, x + w // 2, y, w // 2, h, out)


def partition_frame(width: int, height: int, seed: int, ctu: int = 64) -> np.ndarray:
    """Random QT/BT partition of one frame into blocks with sides 4..64.

    CTUs are ctu x ctu; a partial CTU row or column (2160 = 33*64 + 48) is first
    split into power-of-two strips (48 = 32 + 16).  Returns an int32 array of
    rows (x, y, w, h) covering the frame exactly once.
    """
    rng = _rng(seed)
    out: list = []

    def pow2_parts(n):
        parts, p = [], ctu
        while n > 0:
            while p > n:
                p //= 2
            parts.append(p)
            n -= p
        return parts

    ys, y = [], 0
    for ph in pow2_parts(height):
        ys.append((y, ph))
        y += ph
    xs, x = [], 0
    for pw in pow2_parts(width):
        xs.append((x, pw))
        x += pw
    for (y0, ph) in ys:
        for (x0, pw) in xs:
            _split(rng, x0, y0, pw, ph, out)
    return np.asarray(out, dtype=np.int32)


def frames_workload(nframes: int = 8, width: int = 3840, height: int = 2160,
                    seed: int = SEED_BASE + 3, rho: float = 0.95, sigma: float = 16.0):
    """The batched uneven workload: residual frames, their partitions, and a
    per-block per-axis transform-type draw in {0: DCT-2, 1: adjusted DST-7,
    2: adjusted DCT-8}, uniform.

    Returns (frames int16 [F, H, W], blocks int32 [n, 7] with columns
    (frame, x, y, w, h, type_h, type_v)).
    """
    rng = _rng(seed)
    frames = np.empty((nframes, height, width), np.int16)
    rows = []
    for f in range(nframes):
        fs = int(rng.integers(1 << 31))
        # one AR(1) field per frame, generated in 64-row strips (zero boundary per strip)
        frames[f] = _ar1_field(height, width, rho, sigma, fs)
        part = partition_frame(width, height, fs ^ 0x5A5A)
        types = _rng(fs + 1).integers(0, 3, size=(len(part), 2))
        fcol = np.full((len(part), 1), f, np.int32)
        rows.append(np.concatenate([fcol, part, types.astype(np.int32)], axis=1))
    return frames, np.concatenate(rows, axis=0).astype(np.int32)


def _ar1_field(height, width, rho, sigma, seed, strip=64):
    rng = _rng(seed)
    lw = ar1_filter(width, rho)
    out = np.empty((height, width), np.int16)
    for y0 in range(0, height, strip):
        hh = min(strip, height - y0)
        lh = ar1_filter(hh, rho)
        e = rng.standard_normal((hh, width)) * sigma
        t = lh @ (e @ lw.T)
        out[y0:y0 + hh] = np.clip(np.rint(t), -255, 255).astype(np.int16)
    return out


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# Workload definitions (sizes and model parameters of the five configurations)
WORKLOADS = {
    "cfg1_16x16": dict(nblocks=4096, h=16, w=16, rho=0.90, sigma=20.0, seed=SEED_BASE + 0),
    "cfg2_32x32": dict(nblocks=262144, h=32, w=32, rho=0.95, sigma=16.0, seed=SEED_BASE + 1),
    "cfg3_64x64": dict(nblocks=65536, h=64, w=64, rho=0.97, sigma=12.0, seed=SEED_BASE + 2),
}


def workload_blocks(name: str, nblocks: int | None = None) -> np.ndarray:
    p = dict(WORKLOADS[name])
    if nblocks is not None:
        p["nblocks"] = nblocks
    return ar1_blocks(p["nblocks"], p["h"], p["w"], p["rho"], p["sigma"], p["seed"])


def design_starts(ncand: int, nangles: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """Random starting angles of a batched design search: U[-scale, scale]."""
    return _rng(seed).uniform(-scale, scale, size=(ncand, nangles))
