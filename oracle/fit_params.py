"""Fit and freeze the adjustment parameters (writes the parameter JSON).

The parameter sets the paper used are published only in the JVET documents
it cites (section 3), which are not available, so the parameters are re-fitted
from the paper's own criterion, eq. 2, with the oracle's fitting routines:

  band    K-tap Givens band A before the base (DST-3 in section 2.2; DCT-2 for
          the DCT-2 + band variants), L-BFGS over the angles from theta = 0
  post    B x B sub-block Q after the DCT-2 (section 2.2), Procrustes start
          then weighted L-BFGS

Both the FP64 values and the integer versions round_half_away(2^a x) are
frozen; the GPU library never re-derives integers from angles.  The fit is
non-convex (section 2), so a refit may land elsewhere; parity is defined on
the frozen values.

Run:  python -m oracle.fit_params  [output path]
"""

from __future__ import annotations

import json
import sys
from pathlib import Path

import numpy as np

from . import adjust
from . import transforms as T

A_PREC = 10
OUT = Path(__file__).resolve().parent.parent / "paper_2505_23618_amd" / "params" / "adjust_params.json"

BAND_FITS = ([("S3", "S7", n, k) for n in (4, 8, 16, 32, 64) for k in (4, 6)]
             + [("C2", "S7", 16, 4), ("C2", "S7", 32, 4)])
POST_FITS = [("C2", "S7", n, b) for (n, b) in ((8, 8), (16, 8), (16, 16), (32, 8), (32, 16),
                                               (64, 8), (64, 16))]


def _rows(a):
    return [[float(repr_f) for repr_f in row] for row in np.asarray(a, dtype=np.float64)]


def fit_all():
    entries = []
    for base, target, n, k in BAND_FITS:
        theta, j = adjust.fit_band(base, target, n, k)
        a = adjust.band_matrix(n, k // 2, theta)
        h = adjust.adjusted(base, n, a=a)
        d = T.matrix(target, n)
        corr = [float(abs(h[i] @ d[i])) for i in range(min(8, n))]
        entries.append(dict(
            name=f"band_{base}_{target}_N{n}_K{k}", kind="band", base=base, target=target,
            n=n, taps=k, layers=k // 2, a_prec=A_PREC, criterion=j, low_freq_corr=corr,
            theta=[float(t) for t in theta],
            a_f64=_rows(a), a_int=adjust.round_half_away((1 << A_PREC) * a).tolist()))
        print(f"band {base}->{target} N={n} K={k}: eq2={j:.6f} corr8={min(corr):.4f}", flush=True)
    for base, target, n, b in POST_FITS:
        q, j = adjust.fit_post(base, target, n, b)
        h = adjust.adjusted(base, n, c=adjust.post_matrix(n, q))
        d = T.matrix(target, n)
        corr = [float(abs(h[i] @ d[i])) for i in range(min(8, n))]
        entries.append(dict(
            name=f"post_{base}_{target}_N{n}_B{b}", kind="post", base=base, target=target,
            n=n, block=b, a_prec=A_PREC, criterion=j, low_freq_corr=corr,
            q_f64=_rows(q), q_int=adjust.round_half_away((1 << A_PREC) * q).tolist()))
        print(f"post {base}->{target} N={n} B={b}: eq2={j:.6f} corr8={min(corr):.4f}", flush=True)
    return entries


def main(argv):
    out = Path(argv[1]) if len(argv) > 1 else OUT
    entries = fit_all()
    out.parent.mkdir(parents=True, exist_ok=True)
    with open(out, "w") as f:
        json.dump(dict(a_prec=A_PREC, note="fitted by oracle.fit_params (eq. 2)", entries=entries), f)
    print("wrote", out)


if __name__ == "__main__":
    main(sys.argv)
