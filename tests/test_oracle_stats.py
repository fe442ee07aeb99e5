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
        assert np.abs(q).max() == (32768 + o) // step


def test_half_offset_rounds_half_away_from_zero():
    rng = np.random.Generator(np.random.PCG64(1))
    for step in (2, 6, 64):
        for y in rng.integers(-32768, 32768, 300).tolist() + [step // 2, -step // 2, 3 * step // 2]:
            f = Fraction(y, step)
            want = math.floor(abs(f) + Fraction(1, 2)) * (1 if f >= 0 else -1)
            assert S.quantise(np.array([y]), step, step // 2)[0] == want


def test_exp_golomb_lengths_match_codewords():
    """Order-0 Exp-Golomb: v -> (len(bin(v+1)) - 1) zeros, then bin(v+1)."""
    v = np.arange(0, 40000)
    words = ["0" * (len(bin(k + 1)) - 3) + bin(k + 1)[2:] for k in v.tolist()]
    assert (S.eg0_bits(v) == np.array([len(c) for c in words])).all()
    assert S.eg0_bits(np.array([0, 1, 2, 3, 6, 7, 14])).tolist() == [1, 3, 3, 5, 5, 7, 7]
    # escape suffixes only beyond +-31
    q = np.array([0, 31, -31, 32, -32, 33, 35, -100, 32768])
    assert S.escape_bits(q).tolist() == [0, 0, 0, 1, 1, 3, 5, 13, 29]
    assert S.symbols(q).tolist() == [0, 31, -31, 32, -32, 32, 32, -32, 32]


def _blocks_with_levels(values, h=4, w=4):
    """Blocks whose position 0 runs through `values`; the rest is zero."""
    x = np.zeros((len(values), h, w), np.int16)
    x[:, 0, 0] = values
    return x


@pytest.mark.parametrize("k", [0, 1, 3, 5])
def test_entropy_uniform_over_2k_levels(k):
    vals = np.tile(np.arange(1 << k) - ((1 << k) >> 1), 5)
    st = S.coef_stats(_blocks_with_levels(vals), 1, 0)
    assert st["rate"][0] == pytest.approx(k, abs=1e-12)
    assert (st["rate"][1:] == 0).all() and (st["esc_bits"] == 0).all()


def test_entropy_two_point_closed_forms():
    st = S.coef_stats(_blocks_with_levels([5] * 3 + [-9]), 1, 0)
    assert st["rate"][0] == pytest.approx(0.8112781244591328, abs=1e-12)   # 2 - (3/4) log2 3
    st = S.coef_stats(_blocks_with_levels([0, 1] * 7), 1, 0)
    assert st["rate"][0] == pytest.approx(1.0, abs=1e-12)


def test_escapes_cost_a_symbol_and_their_suffix():
    # half the blocks at level 40 (escape, suffix EG0(8) = 7 bits), half at 0
    st = S.coef_stats(_blocks_with_levels([40, 0] * 6), 1, 0)
    assert st["hist"][0, 64] == 6 and st["hist"][0, 32] == 6
    assert st["esc_bits"][0] == 6 * 7
    assert st["rate"][0] == pytest.approx(1.0 + 3.5, abs=1e-12)
    assert st["summary"]["escape_fraction"] == pytest.approx(6 / (12 * 16))


def test_entropy_of_quantised_gaussian_at_high_rate():
    """H(round(X / step)) -> h(X) - log2 step = 0.5 log2(2 pi e sigma^2) - log2 step
    (sigma / step = 8: escapes, |X| > 31.5 step, have probability 1e-4)."""
    sigma, step = 1024.0, 128        # coarse enough that the integer grid hardly matters
    rng = np.random.Generator(np.random.PCG64(5))
    y = np.clip(np.rint(rng.normal(0.0, sigma, 1 << 20)), -32768, 32767).astype(np.int16)
    st = S.coef_stats(y.reshape(-1, 1, 1), step, step // 2)
    want = 0.5 * math.log2(2 * math.pi * math.e * sigma ** 2) - math.log2(step)
    assert st["rate"][0] == pytest.approx(want, abs=5e-3)
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
    x[:, :2] = np.arange(-40, 40).reshape(1, 2, 40)[:, :, :8] // 2          # some near levels too
    st = S.coef_stats(x, 1, 0)
    y = x.reshape(40, 64).astype(np.int64)
    for p in (0, 9, 17, 63):
        col = y[:, p]
        sym = np.clip(col, -32, 32)
        vals, cnt = np.unique(sym, return_counts=True)
        assert (st["hist"][p, vals + 32] == cnt).all() and st["hist"][p].sum() == 40
        esc = [2 * int(np.floor(np.log2(abs(v) - 31))) + 1 for v in col.tolist() if abs(v) > 31]
        assert st["esc_bits"][p] == sum(esc)
    assert (st["dist"] == 0).all()
    assert st["summary"]["nonzero_fraction"] == np.count_nonzero(y) / y.size


def test_step_beyond_range_zeroes_every_level():
    x = synth.adversarial_blocks(8, 8, "full16", seed=4, n=30)
    x[x == -32768] = 0
    st = S.coef_stats(x, 32768, 0)
    assert (st["hist"][:, 32] == 30).all()
    assert (st["dist"] == st["energy"]).all()
    assert (st["rate"] == 0).all() and st["summary"]["nonzero_fraction"] == 0


def test_brute_force_tiny():
    rng = np.random.Generator(np.random.PCG64(9))
    x = rng.integers(-3000, 3000, size=(7, 4, 8)).astype(np.int16)
    step, o = 24, 11
    st = S.coef_stats(x, step, o)
    for p in range(32):
        col = [int(v) for v in x.reshape(7, 32)[:, p]]
        lev = [(1 if v >= 0 else -1) * ((abs(v) + o) // step) for v in col]
        sym = [max(-32, min(32, l)) for l in lev]
        suffix = 0
        for l in lev:
            if abs(l) > 31:
                k = abs(l) - 32 + 1
                suffix += 2 * (k.bit_length() - 1) + 1
        assert st["energy"][p] == sum(v * v for v in col)
        assert st["dist"][p] == sum((v - l * step) ** 2 for v, l in zip(col, lev))
        for l in set(sym):
            assert st["hist"][p, l + 32] == sym.count(l)
        assert st["esc_bits"][p] == suffix
        h = -sum(sym.count(l) / 7 * math.log2(sym.count(l) / 7) for l in set(sym))
        assert st["rate"][p] == pytest.approx(h + suffix / 7, abs=1e-12)


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
