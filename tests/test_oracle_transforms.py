"""Pins of oracle.transforms against the paper's relations and textbook routines."""

import numpy as np
import pytest
import scipy.fft

from oracle import transforms as T

SIZES = [4, 8, 16, 32, 64]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", T.KINDS)
def test_orthonormal(kind, n):
    m = T.matrix(kind, n)
    assert np.abs(m.T @ m - np.eye(n)).max() < 1e-12
    assert np.abs(m @ m.T - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("n", SIZES)
def test_section21_relations(n):
    # DCT-3 = DCT-2^T, DST-2 = R DCT-2 S, DST-3 = S DCT-2^T R
    c2, r, s = T.dct2(n), T.reversal(n), T.signs(n)
    assert np.abs(T.dct3(n) - c2.T).max() < 1e-13
    assert np.abs(T.dst2(n) - r @ c2 @ s).max() < 1e-13
    assert np.abs(T.dst3(n) - s @ c2.T @ r).max() < 1e-13


@pytest.mark.parametrize("n", SIZES)
def test_eq3_dct8_is_flipped_dst7(n):
    assert np.abs(T.dct8(n) - T.signs(n) @ T.dst7(n) @ T.reversal(n)).max() < 1e-13


@pytest.mark.parametrize("n", SIZES)
def test_eq4_sign_reversal_commute(n):
    assert np.abs(T.signs(n) @ T.dct2(n) - T.dct2(n) @ T.reversal(n)).max() < 1e-13


@pytest.mark.parametrize("n", SIZES)
def test_scipy_dct_dst_types_2_3(n, rng):
    x = rng.standard_normal((5, n))
    for kind, fn, typ in (("C2", scipy.fft.dct, 2), ("C3", scipy.fft.dct, 3),
                          ("S2", scipy.fft.dst, 2), ("S3", scipy.fft.dst, 3)):
        ref = fn(x, type=typ, norm="ortho", axis=-1)
        got = x @ T.matrix(kind, n).T
        assert np.abs(got - ref).max() < 1e-12, kind


@pytest.mark.parametrize("n", SIZES)
def test_dst7_eigenvectors_of_second_difference(n):
    # DST-7 basis = eigenvectors of tridiag(-1, 2, -1) with last diagonal 1,
    # ordered by increasing eigenvalue, first entry positive.
    l = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    l[-1, -1] = 1.0
    w, v = np.linalg.eigh(l)
    v = v[:, np.argsort(w)]
    v = v * np.sign(v[0, :])[None, :]
    assert np.abs(v.T - T.dst7(n)).max() < 1e-12


@pytest.mark.parametrize("n", SIZES)
def test_fast_dct2_equals_dense(n, rng):
    x = rng.standard_normal((7, n))
    assert np.abs(T.dct2_fast(x) - x @ T.dct2(n).T).max() < 1e-12


def test_dct2_dc_row_is_flat():
    for n in SIZES:
        assert np.allclose(T.dct2(n)[0], 1.0 / np.sqrt(n), atol=1e-15)


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_remaining_dsts_orthonormal_and_textbook(n):
    import scipy.fft
    for kind in T.OTHER_DSTS:
        t = T.matrix(kind, n)
        assert np.abs(t @ t.T - np.eye(n)).max() < 1e-12, kind
    eye = np.eye(n)
    # scipy's orthonormal DST-I and DST-IV of the unit vectors are the columns
    assert np.allclose(scipy.fft.dst(eye, type=1, norm="ortho", axis=0), T.dst1(n), atol=1e-13)
    assert np.allclose(scipy.fft.dst(eye, type=4, norm="ortho", axis=0), T.dst4(n), atol=1e-13)
    assert np.allclose(T.dst6(n), T.dst7(n).T, atol=1e-13)
