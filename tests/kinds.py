"""A catalogue of axis kinds for the general-transform tests: every base
(DCT-2, DCT-3, DST-2, DST-3, direct DST-7 / DCT-8), band adjustments with
K = 2, 4, 6, 8 and sub-block adjustments with B = 2, 4, 6, 8, 16 and N / 2,
with and without the DCT-8 flip.  Each kind names the library axis (base,
adjustment, flip, parameter set) and the oracle's axis built from the same
integer and FP64 parameters.  Frozen parameter sets come from the parameter
file; the others are drawn here from random Givens angles (bands) or random
rotation products (sub-blocks), rounded by the oracle's rule."""

from __future__ import annotations

import numpy as np

import paper_2505_23618_amd as ta
from oracle import adjust as OA
from oracle.fixed import Axis

SIZES = (4, 8, 16, 32, 64)
A_PREC = 10


def random_band(n, taps, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    a_f = OA.band_matrix(n, taps // 2, rng.uniform(-0.7, 0.7, OA.n_angles(n, taps // 2)))
    return OA.round_half_away(a_f * (1 << A_PREC)), a_f


def random_post(b, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    q_f = OA.rotation_product(b, rng.uniform(-0.9, 0.9, b * (b - 1) // 2))
    return OA.round_half_away(q_f * (1 << A_PREC)), q_f


# (name, base, adjustment, flip, parameter source) where the source is
# ("frozen", name pattern with {n}) or ("band", K, seed) / ("post", B or "half", seed)
KINDS = [
    ("C2", "C2", "none", False, None),
    ("C3", "C3", "none", False, None),
    ("S2", "S2", "none", False, None),
    ("S3", "S3", "none", False, None),
    ("S7", "S7", "none", False, None),
    ("C8", "C8", "none", False, None),
    ("S7flip", "S7", "none", True, None),
    ("S3band4", "S3", "band", False, ("frozen", "band_S3_S7_N{n}_K4")),
    ("S3band4flip", "S3", "band", True, ("frozen", "band_S3_S7_N{n}_K4")),
    ("S3band6", "S3", "band", False, ("frozen", "band_S3_S7_N{n}_K6")),
    ("S3band6flip", "S3", "band", True, ("frozen", "band_S3_S7_N{n}_K6")),
    ("C3band2", "C3", "band", False, ("band", 2, 11)),
    ("S2band8", "S2", "band", False, ("band", 8, 12)),
    ("C2band8flip", "C2", "band", True, ("band", 8, 13)),
    ("C2post8", "C2", "post", False, ("frozen", "post_C2_S7_N{n}_B8")),
    ("C2post8flip", "C2", "post", True, ("frozen", "post_C2_S7_N{n}_B8")),
    ("C2post16", "C2", "post", False, ("frozen", "post_C2_S7_N{n}_B16")),
    ("C2post16flip", "C2", "post", True, ("frozen", "post_C2_S7_N{n}_B16")),
    ("S3post4", "S3", "post", False, ("post", 4, 21)),
    ("C3post2flip", "C3", "post", True, ("post", 2, 22)),
    ("S2post6", "S2", "post", False, ("post", 6, 23)),
    ("C2posthalf", "C2", "post", False, ("post", "half", 24)),
]


def min_size(kind) -> int:
    src = kind[4]
    if src is None:
        return 4
    if src[0] == "frozen":
        return 16 if "B16" in src[1] else 8 if "B8" in src[1] else 4
    if src[0] == "post" and src[1] != "half":
        return max(4, 1 << int(np.ceil(np.log2(src[1]))))
    return 4


def kinds_for(n: int):
    """Indices of the kinds that exist at size n."""
    return [i for i, k in enumerate(KINDS) if min_size(k) <= n]


class Catalogue:
    """Registers every kind at every size it exists at with a context:
    axis id 100 + 5 * kind + log2(n) - 2, parameter sets from id 100 on."""

    def __init__(self, ctx, frozen_ids: dict, params: dict):
        self.ctx, self.params = ctx, params
        self.axis = {}
        self.oracle = {}
        pid = 100
        for i, (name, base, adj, flip, src) in enumerate(KINDS):
            for n in SIZES:
                if min_size(KINDS[i]) > n:
                    continue
                aid = 100 + 5 * i + int(np.log2(n)) - 2
                lib_adj = {"none": ta.ADJ_NONE, "band": ta.ADJ_BAND, "post": ta.ADJ_POST}[adj]
                if adj == "none":
                    ctx.axis(aid, ta.BASES[base], ta.ADJ_NONE, flip, 0)
                    oax = Axis(base=base, adj="none", flip=flip)
                else:
                    if src[0] == "frozen":
                        pname = src[1].format(n=n)
                        e = params[pname]
                        use = frozen_ids[pname]
                        if adj == "band":
                            m_int, m_f = np.asarray(e["a_int"], np.int64), np.asarray(e["a_f64"])
                        else:
                            m_int, m_f = np.asarray(e["q_int"], np.int64), np.asarray(e["q_f64"])
                    else:
                        use = pid
                        pid += 1
                        if src[0] == "band":
                            m_int, m_f = random_band(n, src[1], src[2] * 100 + n)
                            ctx.set_band(use, m_int, m_f, src[1])
                        else:
                            b = n // 2 if src[1] == "half" else src[1]
                            m_int, m_f = random_post(b, src[2] * 100 + n)
                            ctx.set_post(use, m_int, m_f, n)
                    ctx.axis(aid, ta.BASES[base], lib_adj, flip, use)
                    if adj == "band":
                        oax = Axis(base=base, adj="band", flip=flip, a_int=m_int, a_f=m_f)
                    else:
                        oax = Axis(base=base, adj="post", flip=flip, q_int=m_int, q_f=m_f)
                self.axis[(i, n)] = aid
                self.oracle[(i, n)] = oax
