"""Statistics of quantised transform coefficients: a codec-free proxy for the
coding results of the paper's experiments section (test infrastructure only).

The paper judges the adjusted transforms by their all-intra BD-rate inside a
video codec (Tables 2 and 3): whether replacing the DST-7 / DCT-8 by their
adjusted approximations changes compression.  Without the codec and its test
sequences, the same question is asked of the coefficients directly: on the
same residual blocks, how do energy compaction and the rate of the quantised
coefficients compare between the adjusted and the exact transforms?
Definitions (this module's reading; the paper prints none of them):

  quantiser     level q = sign(y) * floor((|y| + o) / step), integer step >= 1
                and rounding offset 0 <= o < step (o = step // 2 rounds to the
                nearest level, ties away from zero); reconstruction q * step
  symbol        s = q for |q| <= 31, else +32 or -32 (an escape of that sign):
                65 symbols, as a codec sends small levels with adaptive
                entropy coding and large ones as an escape plus a suffix
  histogram     per coefficient position p (row-major, p = row * W + col),
                the count of every symbol over the blocks (column 32 + s)
  escape bits   per position, the sum over escapes of the length of the
                order-0 Exp-Golomb code of |q| - 32: 2 floor(log2(|q| - 31)) + 1
  rate          R_p = H_p + escape bits_p / n, where H_p is the first-order
                entropy (bits) of the symbols at position p over n blocks;
                the rate proxy is the mean of R_p over the H*W positions
  energy        E_p = sum over blocks of y_p^2 (second moment: the residuals
                are zero-mean by construction)
  distortion    D_p = sum over blocks of (y_p - q_p step)^2
  coding gain   10 log10(arithmetic mean / geometric mean) of the per-position
                mean energies E_p / n: the transform coding gain
  low band      fraction of the energy in the top-left (H/4) x (W/4)
                positions, the region the sub-block adjustment acts on

Integer results (histograms, escape bits, energies, distortions) are exact
in int64; rates and the summary are FP64.  With no blocks every output is
zero; with no energy the coding gain and the low-band fraction are 0, and a
zero energy at some positions only makes the coding gain +inf.

Pins (tests/test_oracle_stats.py): the quantiser against exact rational
rounding on every input in range; the Exp-Golomb lengths against codewords
built bit by bit; entropies of constructed distributions with closed forms
(uniform over 2^k levels, two-point); the high-rate entropy of a quantised
Gaussian against its differential entropy minus log2(step); the coding gain
of the eigenvalues of the AR(1) covariance against the determinant closed
form, in 1-D and separably in 2-D; the degenerate quantisers (step 1:
identity, no distortion; step beyond the range: all levels zero, distortion
equals energy); brute-force sums on tiny inputs; and, on AR(1) residuals,
the ordering exact DST-7 > adjusted > DCT-2 in coding gain and rate.
"""

from __future__ import annotations

import numpy as np

NEAR = 31                      # |levels| sent as their own symbol
NSYM = 2 * NEAR + 3            # -32 (escape), -31..31, +32 (escape)
SUMMARY = ("bits_per_coef", "mse_per_coef", "energy_per_coef", "coding_gain_db",
           "low_band_fraction", "nonzero_fraction", "escape_fraction")


def quantise(y: np.ndarray, step: int, offset: int) -> np.ndarray:
    """q = sign(y) floor((|y| + o) / step), in int64."""
    if not (1 <= step and 0 <= offset < step):
        raise ValueError("need step >= 1 and 0 <= offset < step")
    a = np.abs(np.asarray(y, dtype=np.int64))
    q = (a + offset) // step
    return np.where(np.asarray(y) < 0, -q, q)


def symbols(q: np.ndarray) -> np.ndarray:
    """Levels beyond +-31 become the escape symbols +-32."""
    return np.clip(q, -(NEAR + 1), NEAR + 1)


def eg0_bits(v: np.ndarray) -> np.ndarray:
    """Length of the order-0 Exp-Golomb codeword of v >= 0: 2 floor(log2(v+1)) + 1."""
    v = np.asarray(v, dtype=np.int64)
    return 2 * (np.floor(np.log2(v + 1)).astype(np.int64)) + 1


def escape_bits(q: np.ndarray) -> np.ndarray:
    """Suffix bits of every level: Exp-Golomb of |q| - 32 for escapes, else 0."""
    a = np.abs(np.asarray(q, dtype=np.int64))
    return np.where(a > NEAR, eg0_bits(np.maximum(a - (NEAR + 1), 0)), 0)


def entropy_bits(counts: np.ndarray) -> float:
    """First-order entropy in bits of a histogram (zero bins contribute 0)."""
    c = np.asarray(counts, dtype=np.float64)
    n = c.sum()
    if n == 0:
        return 0.0
    p = c[c > 0] / n
    return float(-(p * np.log2(p)).sum())


def coding_gain_db(energies: np.ndarray) -> float:
    """10 log10(AM / GM) of a set of per-position energies (variances)."""
    e = np.asarray(energies, dtype=np.float64).ravel()
    with np.errstate(divide="ignore", invalid="ignore"):
        am = e.mean()
        gm = np.exp2(np.log2(e).mean())
        return float(10.0 * np.log10(am / gm))


def coef_stats(coef: np.ndarray, step: int, offset: int) -> dict:
    """All statistics of a batch of coefficient blocks (nblocks, H, W) int16.

    Returns hist (P, 65) int64 with column 32 + s counting symbol s, escape
    bits, energy and dist (P,) int64, rate (P,) float64, and the summary dict
    with the fields of SUMMARY.
    """
    coef = np.asarray(coef)
    nb, h, w = coef.shape
    p = h * w
    y = coef.reshape(nb, p).astype(np.int64)
    q = quantise(y, step, offset)
    s = symbols(q)
    hist = np.zeros((p, NSYM), dtype=np.int64)
    for k in range(p):
        hist[k] = np.bincount(s[:, k] + NEAR + 1, minlength=NSYM)
    esc = escape_bits(q).sum(axis=0)
    energy = (y * y).sum(axis=0)
    d = y - q * step
    dist = (d * d).sum(axis=0)
    rate = np.array([entropy_bits(hist[k]) + (esc[k] / nb if nb else 0.0) for k in range(p)])
    if nb == 0:
        summary = dict.fromkeys(SUMMARY, 0.0)
    else:
        ncoef = float(nb) * p
        low = np.zeros((h, w), dtype=bool)
        low[: h // 4, : w // 4] = True
        etot = float(energy.sum())
        summary = {
            "bits_per_coef": float(rate.mean()),
            "mse_per_coef": float(dist.sum()) / ncoef,
            "energy_per_coef": etot / ncoef,
            "coding_gain_db": coding_gain_db(energy / nb) if etot > 0 else 0.0,
            "low_band_fraction": float(energy[low.ravel()].sum()) / etot if etot > 0 else 0.0,
            "nonzero_fraction": float(np.count_nonzero(q)) / ncoef,
            "escape_fraction": float(np.count_nonzero(np.abs(q) > NEAR)) / ncoef,
        }
    return {"hist": hist, "esc_bits": esc, "energy": energy, "dist": dist, "rate": rate, "summary": summary}
