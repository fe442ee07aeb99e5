"""Pins of the oracle's quantised-coefficient statistics (the coding-gain
proxy for the coding results, Tables 2 and 3): every quantity is checked
against something the mathematics fixes, not against the oracle itself."""

import math
from fractions import Fraction

import numpy as np
import pytest

import paper_2505_23618_amd as ta
import synth
from oracle import fixed as F
from oracle import stats as S
from tests.libcases import oracle_axis

ALL16 = np.arange(-32768, 32768, dtype=np.int64)


@pytest.mark.parametrize("step", [1, 2, 3, 7, 32, 100, 32768])
def test_quantiser_is_floor_of_offset_magnitude(step):
    """Every int16 input: step |q| <= |y| + o < step (|q| + 1), sign of q that of y."""
    for o in sorted({0, step // 2, step - 1}):
        q = S.quantise(ALL16, step, o)
        a = np.abs(ALL16)
        assert (step * np.abs(q) <= a + o).all() and (a + o < step * (np.abs(q) + 1)).all()
        assert ((q == 0) | (np.sign(q) == np.sign(ALL16))).all()
        assert np.abs(q).max() == S.max_level(step, o)


def test_half_offset_rounds_half_away_from_zero():
    rng = np.random.Generator(np.random.PCG64(1))
    for step in (2, 6, 64):
        for y in rng.integers(-32768, 32768, 300).tolist() + [step // 2, -step // 2, 3 * step // 2]:
            f = Fraction(y, step)
            want = math.floor(abs(f) + Fraction(1, 2)) * (1 if f >= 0 else -1)
            assert S.quantise(np.array([y]), step, step // 2)[0] == want


def _blocks_with_levels(values, h=4, w=4):
    """Blocks whose position 0 runs through `values`; the rest is zero."""
    x = np.zeros((len(values), h, w), np.int16)
    x[:, 0, 0] = values
    return x


@pytest.mark.parametrize("k", [0, 1, 3, 6])
def test_entropy_uniform_over_2k_levels(k):
    vals = np.tile(np.arange(1 << k) - ((1 << k) >> 1), 5)
    st = S.coef_stats(_blocks_with_levels(vals), 1, 0)
    assert st["entropy"][0] == pytest.approx(k, abs=1e-12)
    assert (st["entropy"][1:] == 0).all()


def test_entropy_two_point_closed_forms():
    st = S.coef_stats(_blocks_with_levels([5] * 3 + [-9]), 1, 0)
    assert st["entropy"][0] == pytest.approx(0.8112781244591328, abs=1e-12)   # 2 - (3/4) log2 3
    st = S.coef_stats(_blocks_with_levels([0, 1] * 7), 1, 0)
    assert st["entropy"][0] == pytest.approx(1.0, abs=1e-12)


def test_entropy_of_quantised_gaussian_at_high_rate():
    """H(round(X / step)) -> h(X) - log2 step = 0.5 log2(2 pi e sigma^2) - log2 step."""
    sigma, step = 400.0, 16
    rng = np.random.Generator(np.random.PCG64(5))
    y = np.clip(np.rint(rng.normal(0.0, sigma, 1 << 20)), -32768, 32767).astype(np.int16)
    st = S.coef_stats(y.reshape(-1, 1, 1), step, step // 2)
    want = 0.5 * math.log2(2 * math.pi * math.e * sigma ** 2) - math.log2(step)
    assert st["entropy"][0] == pytest.approx(want, abs=5e-3)
    # uniform quantisation noise: step^2 / 12 per coefficient
    assert st["summary"]["mse_per_coef"] == pytest.approx(step ** 2 / 12, rel=2e-2)


@pytest.mark.parametrize("n,rho", [(8, 0.9), (32, 0.95)])
def test_coding_gain_of_ar1_klt_matches_determinant(n, rho):
    """The KLT of a unit-variance AR(1) source has variances = eigenvalues of
    the Toeplitz covariance rho^|i-j|; their mean is 1 and their product is
    det = (1 - rho^2)^(n-1), so the gain is -10 (n-1)/n log10(1 - rho^2).
    The separable 2-D source has eigenvalues l_i l_j: twice the 1-D gain."""
    r = rho ** np.abs(np.subtract.outer(np.arange(n), np.arange(n)))
    lam = np.linalg.eigvalsh(r)
    want = -10.0 * (n - 1) / n * math.log10(1 - rho * rho)
    assert S.coding_gain_db(lam) == pytest.approx(want, abs=1e-9)
    assert S.coding_gain_db(np.outer(lam, lam)) == pytest.approx(2 * want, abs=1e-9)
    assert S.coding_gain_db(np.ones(n)) == pytest.approx(0.0, abs=1e-12)


def test_step_one_is_identity_without_distortion():
    x = synth.adversarial_blocks(8, 8, "full16", seed=3, n=40)
    st = S.coef_stats(x, 1, 0)
    lv = S.max_level(1, 0)
    y = x.reshape(40, 64).astype(np.int64)
    for p in (0, 17, 63):
        vals, cnt = np.unique(y[:, p], return_counts=True)
        assert (st["hist"][p, vals + lv] == cnt).all() and st["hist"][p].sum() == 40
    assert (st["dist"] == 0).all()
    assert st["summary"]["nonzero_fraction"] == np.count_nonzero(y) / y.size


def test_step_beyond_range_zeroes_every_level():
    x = synth.adversarial_blocks(8, 8, "full16", seed=4, n=30)
    x[x == -32768] = 0
    st = S.coef_stats(x, 32768, 0)
    assert S.max_level(32768, 0) == 1
    assert (st["hist"][:, 1] == 30).all()
    assert (st["dist"] == st["energy"]).all()
    assert (st["entropy"] == 0).all() and st["summary"]["nonzero_fraction"] == 0


def test_brute_force_tiny():
    rng = np.random.Generator(np.random.PCG64(9))
    x = rng.integers(-300, 300, size=(7, 4, 8)).astype(np.int16)
    step, o = 24, 11
    st = S.coef_stats(x, step, o)
    lv = S.max_level(step, o)
    for p in range(32):
        col = [int(v) for v in x.reshape(7, 32)[:, p]]
        lev = [(1 if v >= 0 else -1) * ((abs(v) + o) // step) for v in col]
        assert st["energy"][p] == sum(v * v for v in col)
        assert st["dist"][p] == sum((v - l * step) ** 2 for v, l in zip(col, lev))
        for l in set(lev):
            assert st["hist"][p, l + lv] == lev.count(l)
        h = -sum(lev.count(l) / 7 * math.log2(lev.count(l) / 7) for l in set(lev))
        assert st["entropy"][p] == pytest.approx(h, abs=1e-12)


def test_low_band_fraction_and_degenerate_summaries():
    x = np.zeros((3, 16, 16), np.int16)
    x[:, :4, :4] = 7
    assert S.coef_stats(x, 4, 2)["summary"]["low_band_fraction"] == 1.0
    assert S.coef_stats(x, 4, 2)["summary"]["coding_gain_db"] == math.inf
    x = np.zeros((3, 16, 16), np.int16)
    x[:, 4:, :] = -3
    assert S.coef_stats(x, 4, 2)["summary"]["low_band_fraction"] == 0.0
    z = S.coef_stats(np.zeros((5, 8, 8), np.int16), 4, 2)["summary"]
    assert z["coding_gain_db"] == 0.0 and z["low_band_fraction"] == 0.0 and z["bits_per_coef"] == 0.0
    e = S.coef_stats(np.zeros((0, 8, 8), np.int16), 4, 2)
    assert all(v == 0.0 for v in e["summary"].values()) and e["hist"].sum() == 0


def test_adjusted_transforms_sit_between_dct2_and_dst7_on_ar1_residuals():
    """On AR(1) residuals with zero top/left boundary the DST-7 compacts
    energy better than the DCT-2, and the adjusted DST-7 approximations
    recover most of that advantage (the 6-tap band more than the 4-tap)."""
    params = ta.load_param_file()
    x = synth.ar1_blocks(400, 32, 32, 0.95, 16.0, seed=8)
    specs = {"C2": (ta.DCT2, ta.ADJ_NONE, False, None), "S7": (ta.DST7, ta.ADJ_NONE, False, None),
             "K4": (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N32_K4"),
             "K6": (ta.DST3, ta.ADJ_BAND, False, "band_S3_S7_N32_K6"),
             "B8": (ta.DCT2, ta.ADJ_POST, False, "post_C2_S7_N32_B8")}
    gain, bits = {}, {}
    for k, spec in specs.items():
        ax = oracle_axis(params, *spec)
        s = S.coef_stats(F.fwd2d(x, ax, ax), 64, 32)["summary"]
        gain[k], bits[k] = s["coding_gain_db"], s["bits_per_coef"]
    for k in ("K4", "K6", "B8"):
        assert gain["C2"] + 0.1 < gain[k] < gain["S7"]
        assert bits["S7"] < bits[k] < bits["C2"]
        assert gain["S7"] - gain[k] < 0.5 * (gain["S7"] - gain["C2"])
    assert gain["K6"] > gain["K4"]
