"""Pins of oracle.fp (FP64 2-D path) and of the synthetic input generators."""

import numpy as np
import pytest
import scipy.fft

import synth
from oracle import fp as P
from tests import cfgs


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_plain_dct2_2d_equals_scipy(n, rng):
    x = rng.standard_normal((3, n, n))
    ax = cfgs.plain_axis("C2")
    ref = scipy.fft.dctn(x, type=2, norm="ortho", axes=(1, 2))
    assert np.abs(P.fwd2d(x, ax, ax) - ref).max() < 1e-11


def test_rectangular_mixed_dst2_dct3_equals_scipy(rng):
    x = rng.standard_normal((2, 8, 32))           # H = 8, W = 32
    got = P.fwd2d(x, cfgs.plain_axis("S2"), cfgs.plain_axis("C3"))
    ref = scipy.fft.dct(scipy.fft.dst(x, type=2, norm="ortho", axis=2), type=3, norm="ortho", axis=1)
    assert np.abs(got - ref).max() < 1e-11


@pytest.mark.parametrize("which", ["cfg1", "cfg2", "cfg3"])
def test_roundtrip_and_kronecker(params, which, rng):
    ax_h, ax_v = {"cfg1": cfgs.cfg1, "cfg2": cfgs.cfg2, "cfg3": cfgs.cfg3}[which](params)
    n = {"cfg1": 16, "cfg2": 32, "cfg3": 64}[which]
    x = rng.standard_normal((2, n, n))
    y = P.fwd2d(x, ax_h, ax_v)
    assert np.abs(P.inv2d(y, ax_h, ax_v) - x).max() < 1e-12
    hh, hv = P.axis_matrix(ax_h, n), P.axis_matrix(ax_v, n)
    k = np.kron(hv, hh)
    assert np.abs(y[0].reshape(-1) - k @ x[0].reshape(-1)).max() < 1e-11


def test_energy_preserved(params, rng):
    ax_h, ax_v = cfgs.cfg3(params)
    x = rng.standard_normal((2, 64, 64))
    y = P.fwd2d(x, ax_h, ax_v)
    assert abs(np.sum(y ** 2) - np.sum(x ** 2)) < 1e-9 * np.sum(x ** 2)


# ---------------------------------------------------------------------------
# synthetic inputs
# ---------------------------------------------------------------------------

def test_ar1_prefix_property_and_range():
    a = synth.ar1_blocks(20, 32, 32, 0.95, 16.0, seed=5)
    b = synth.ar1_blocks(50, 32, 32, 0.95, 16.0, seed=5, chunk=7)
    assert (a == b[:20]).all()
    assert a.dtype == np.int16 and np.abs(a).max() <= 255


def test_ar1_correlation_matches_rho():
    x = synth.ar1_blocks(400, 32, 32, 0.9, 1.0, seed=1).astype(np.float64)
    # interior lag-1 correlation along rows approaches rho for a stationary-ish AR(1)
    a, b = x[:, 16:, 16:-1].ravel(), x[:, 16:, 17:].ravel()
    r = np.corrcoef(a, b)[0, 1]
    assert 0.85 < r < 0.93


def test_partition_covers_frame_exactly():
    part = synth.partition_frame(384, 216, seed=3)
    cover = np.zeros((216, 384), np.int32)
    for x, y, w, h in part:
        assert w in (4, 8, 16, 32, 64) and h in (4, 8, 16, 32, 64)
        cover[y:y + h, x:x + w] += 1
    assert (cover == 1).all()
