"""Logical transform configurations of the five workloads, as oracle axes.

Test helper: turns the frozen parameter JSON into ``oracle.fixed.Axis``
objects.  The GPU side receives the same parameters through the library's
own C-ABI; nothing here is shared with it beyond the parameter values.
"""

import numpy as np

from oracle.fixed import Axis


def band_axis(params, base, n, taps, flip=False, fit_base=None):
    e = params[f"band_{fit_base or base}_S7_N{n}_K{taps}"]
    return Axis(base=base, adj="band", flip=flip, a_int=np.asarray(e["a_int"], np.int64),
                a_f=np.asarray(e["a_f64"]))


def post_axis(params, n, b, flip=False):
    e = params[f"post_C2_S7_N{n}_B{b}"]
    return Axis(base="C2", adj="post", flip=flip, q_int=np.asarray(e["q_int"], np.int64),
                q_f=np.asarray(e["q_f64"]))


def plain_axis(base, flip=False):
    return Axis(base=base, adj="none", flip=flip)


def cfg1(params):
    a = band_axis(params, "C2", 16, 4)
    return a, a


def cfg2(params, taps=4):
    a = band_axis(params, "S3", 32, taps)
    return a, a


def cfg3(params):
    # rows (horizontal): DCT-8 by eq. 5; columns (vertical): DST-7
    return post_axis(params, 64, 16, flip=True), post_axis(params, 64, 16, flip=False)


def type_axis(params, t, n):
    """Batched workload types: 0 DCT-2, 1 adjusted DST-7, 2 adjusted DCT-8
    (DST-3 + 4-tap band, fitted per size)."""
    if t == 0:
        return plain_axis("C2")
    return band_axis(params, "S3", n, 4, flip=(t == 2))
