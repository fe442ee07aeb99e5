"""Host-side setup of the GPU design study: the package's transform matrices
and candidate signs equal the oracle's (no GPU needed)."""

import numpy as np
import pytest

from oracle import design as Dz
from oracle import transforms as T
from paper_2505_23618_amd import design as PD


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_matrices_match_oracle(n):
    for kind in PD.BASES + PD.TARGETS:
        assert np.abs(PD.transform_matrix(kind, n) - T.matrix(kind, n)).max() < 1e-14, kind


def test_study_candidates_and_signs():
    mats, cands, labels = PD.study(8, 3)
    assert cands.shape == (len(PD.BASES) * len(PD.TARGETS) * 2 * 3, 4)
    for row, (bk, tk, mode) in zip(cands, labels):
        assert PD.BASES[row[0]] == bk and (PD.BASES + PD.TARGETS)[row[1]] == tk
        assert row[2] == PD.MODES.index(mode)
        assert row[3] == Dz.sigma_for(T.matrix(bk, 8), T.matrix(tk, 8), mode)
