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


def _second_difference(n):
    return 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def _eig_rows(l):
    """Eigenvectors of a symmetric matrix as rows, by ascending eigenvalue,
    each signed so that its first entry is positive."""
    w, v = np.linalg.eigh(l)
    order = np.argsort(w)
    v = v[:, order]
    return w[order], (v * np.sign(v[0, :])[None, :]).T


@pytest.mark.parametrize("n", SIZES)
def test_dst5_eigenvectors_of_second_difference(n):
    # A sampled sinusoid s(i) = sin(w (i + 1)) meets the interior rows of
    # tridiag(-1, 2, -1) with eigenvalue 2 - 2 cos w.  DST-5 takes
    # w = 2 pi (k + 1) / (2N + 1): s(-1) = 0 (Dirichlet at the left, first row
    # unchanged) and w (2N + 1) = 2 pi (k + 1) gives s(N) = -s(N - 1), so the
    # last row reads -s(N-2) + 3 s(N-1): last diagonal entry 3.  The N values
    # of w are distinct, so each row is fixed up to its sign (s(0) > 0).
    l = _second_difference(n)
    l[-1, -1] = 3.0
    w, rows = _eig_rows(l)
    k = np.arange(n)
    assert np.abs(w - (2 - 2 * np.cos(2 * np.pi * (k + 1) / (2 * n + 1)))).max() < 1e-12
    assert np.abs(rows - T.dst5(n)).max() < 1e-12


@pytest.mark.parametrize("n", SIZES)
def test_dst8_eigenvectors_of_second_difference(n):
    # DST-8 samples s(i) = sin(w (i + 1/2)) with w = pi (2k + 1) / (2N - 1).
    # Left: s(-1) = -s(0), so the first row reads 3 s(0) - s(1).  Right:
    # w (N - 1/2) = (2k + 1) pi / 2 puts a peak at i = N - 1, so s(N) = s(N - 2)
    # and the last row reads -2 s(N-2) + 2 s(N-1).  Scaling the last sample by
    # 1/sqrt2 (the f_{N-1} of the definition) makes the matrix symmetric:
    # the last off-diagonal pair becomes -sqrt2.
    l = _second_difference(n)
    l[0, 0] = 3.0
    l[-1, -2] = l[-2, -1] = -np.sqrt(2.0)
    w, rows = _eig_rows(l)
    k = np.arange(n)
    assert np.abs(w - (2 - 2 * np.cos(np.pi * (2 * k + 1) / (2 * n - 1)))).max() < 1e-12
    assert np.abs(rows - T.dst8(n)).max() < 1e-12


def test_dst5_dst8_hand_values_n4():
    # N = 4 entries evaluated by hand from the sinusoids: DST-5 row 0 is
    # (2/3) sin(2 pi (i + 1) / 9), DST-8 row 0 is sqrt(4/7) sin(pi (2i + 1) / 14)
    # with the last entry divided by sqrt2 (row k = 0 is not the scaled row).
    s5 = T.dst5(4)
    assert np.allclose(s5[0], [2 / 3 * np.sin(2 * np.pi * j / 9) for j in (1, 2, 3, 4)], atol=1e-15)
    s8 = T.dst8(4)
    ref = [np.sqrt(4 / 7) * np.sin(np.pi * j / 14) for j in (1, 3, 5, 7)]
    ref[3] /= np.sqrt(2)
    assert np.allclose(s8[0], ref, atol=1e-15)
    # the last row k = 3 carries the 1/sqrt2 on every entry and 1/2 on the corner
    ref3 = [np.sqrt(4 / 7) * np.sin(7 * np.pi * j / 14) / np.sqrt(2) for j in (1, 3, 5, 7)]
    ref3[3] /= np.sqrt(2)
    assert np.allclose(s8[3], ref3, atol=1e-15)
