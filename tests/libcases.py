"""Transform cases shared by the GPU parity tests and the benchmark's checks.

Each case names a block size and the per-axis transform twice: once as a
library axis (base, adjustment, flip, parameter set) registered through the
C ABI, once as the oracle's axis built from the same frozen parameters.
"""

import numpy as np

import paper_2505_23618_amd as ta
from oracle.fixed import Axis


def oracle_axis(params, base, adj, flip, pname):
    if adj == ta.ADJ_BAND:
        e = params[pname]
        return Axis(base=_name(base), adj="band", flip=flip, a_int=np.asarray(e["a_int"], np.int64),
                    a_f=np.asarray(e["a_f64"]))
    if adj == ta.ADJ_POST:
        e = params[pname]
        return Axis(base=_name(base), adj="post", flip=flip, q_int=np.asarray(e["q_int"], np.int64),
                    q_f=np.asarray(e["q_f64"]))
    return Axis(base=_name(base), adj="none", flip=flip)


def _name(base):
    return {v: k for k, v in ta.BASES.items()}[base]


# name: (W, H, horizontal spec, vertical spec); spec = (base, adj, flip, param name)
S3B4_32 = (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N32_K4")
CASES = {
    "cfg2_dst7_k4": (32, 32, S3B4_32, S3B4_32),
    "cfg2_dct8_k4": (32, 32, (ta.DST3, ta.ADJ_BAND, True, "band_S3_S7_N32_K4"),
                     (ta.DST3, ta.ADJ_BAND, True, "band_S3_S7_N32_K4")),
    "cfg2_dst7_k6": (32, 32, (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N32_K6"),
                     (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N32_K6")),
    "direct_dst7_32": (32, 32, (ta.DST7, ta.ADJ_NONE, False, None), (ta.DST7, ta.ADJ_NONE, False, None)),
    "dct2_32": (32, 32, (ta.DCT2, ta.ADJ_NONE, False, None), (ta.DCT2, ta.ADJ_NONE, False, None)),
    "direct_dct8_32": (32, 32, (ta.DCT8, ta.ADJ_NONE, False, None), (ta.DCT8, ta.ADJ_NONE, False, None)),
    "post8_32": (32, 32, (ta.DCT2, ta.ADJ_POST, False, "post_C2_S7_N32_B8"),
                 (ta.DCT2, ta.ADJ_POST, True, "post_C2_S7_N32_B8")),
    "cfg1_dct2_band_16": (16, 16, (ta.DCT2, ta.ADJ_BAND, False, "band_C2_S7_N16_K4"),
                          (ta.DCT2, ta.ADJ_BAND, False, "band_C2_S7_N16_K4")),
    "cfg3_post16_64": (64, 64, (ta.DCT2, ta.ADJ_POST, True, "post_C2_S7_N64_B16"),
                       (ta.DCT2, ta.ADJ_POST, False, "post_C2_S7_N64_B16")),
    "direct_dst7_64": (64, 64, (ta.DST7, ta.ADJ_NONE, False, None), (ta.DST7, ta.ADJ_NONE, False, None)),
    "band4_64": (64, 64, (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N64_K4"),
                 (ta.DST3, ta.ADJ_BAND, True, "band_S3_S7_N64_K4")),
    "band6_64": (64, 64, (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N64_K6"),
                 (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N64_K6")),
    "post8_64": (64, 64, (ta.DCT2, ta.ADJ_POST, True, "post_C2_S7_N64_B8"),
                 (ta.DCT2, ta.ADJ_POST, False, "post_C2_S7_N64_B8")),
    "dst7_band_4": (4, 4, (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N4_K4"),
                    (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N4_K4")),
    "dst3_dct3_8": (8, 8, (ta.DST3, ta.ADJ_NONE, False, None), (ta.DCT3, ta.ADJ_NONE, False, None)),
    "dst2_dct8_16x8": (16, 8, (ta.DST2, ta.ADJ_NONE, False, None), (ta.DCT8, ta.ADJ_NONE, False, None)),
    "dct2_dst7band_8x32": (8, 32, (ta.DCT2, ta.ADJ_NONE, False, None), S3B4_32),
}

# cases built only for the fp32 kernels
F32_ONLY = {
    "dst2_dct8_8x16": (8, 16, (ta.DST2, ta.ADJ_NONE, False, None), (ta.DCT8, ta.ADJ_NONE, False, None)),
}
ALL_CASES = {**CASES, **F32_ONLY}


class Registered:
    """A context with every frozen parameter set and every case's axes."""

    def __init__(self, device=0, bit_depth=8):
        self.ctx = ta.Context(device, bit_depth=bit_depth)
        self.ids = ta.load_params(self.ctx)
        self.params = ta.load_param_file()
        self.axes = {}
        nxt = 0
        for name, (w, h, sh, sv) in ALL_CASES.items():
            pair = []
            for spec in (sh, sv):
                base, adj, flip, pname = spec
                aid = nxt
                nxt += 1
                self.ctx.axis(aid, base, adj, flip, self.ids[pname] if pname else 0)
                pair.append(aid)
            self.axes[name] = tuple(pair)

    def oracle_axes(self, name):
        w, h, sh, sv = ALL_CASES[name]
        return (oracle_axis(self.params, *sh), oracle_axis(self.params, *sv))
