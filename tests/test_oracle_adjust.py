"""Pins of oracle.adjust: structure, gradients and the closed-form special case."""

import numpy as np
import pytest

from oracle import adjust
from oracle import transforms as T


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("taps", [4, 6])
def test_band_orthogonal_and_sparse(n, taps, rng):
    layers = taps // 2
    th = rng.uniform(-1, 1, adjust.n_angles(n, layers))
    a = adjust.band_matrix(n, layers, th)
    assert np.abs(a.T @ a - np.eye(n)).max() < 1e-12
    nnz = (np.abs(a) > 1e-14).sum(axis=1)
    assert nnz.max() <= taps
    # every row of A and of A^T lies in an aligned window of `taps` columns
    for m in (a, a.T):
        for i, row in enumerate(m):
            idx = np.nonzero(np.abs(row) > 1e-14)[0]
            assert idx.max() - idx.min() < taps


def test_angle_counts():
    # 2 layers on 32 points: 16 even pairs + 15 odd pairs = 31 angles
    assert adjust.n_angles(32, 2) == 31
    assert adjust.n_angles(32, 3) == 47
    assert adjust.n_angles(4, 2) == 3


def test_zero_angles_give_base():
    for base in ("C2", "S3"):
        h = adjust.adjusted(base, 16, a=adjust.band_matrix(16, 2, np.zeros(15)))
        assert np.abs(h - T.matrix(base, 16)).max() == 0.0


def _num_grad(f, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("base,n,taps", [("S3", 16, 4), ("C2", 8, 6), ("S3", 32, 4)])
def test_band_gradient_matches_central_differences(base, n, taps, rng):
    layers = taps // 2
    th = rng.uniform(-0.5, 0.5, adjust.n_angles(n, layers))
    bm, d, w = T.matrix(base, n), T.dst7(n), adjust.weights(n)
    f = lambda t: adjust.band_objective(t, bm, d, n, layers, w)[0]
    g = adjust.band_objective(th, bm, d, n, layers, w)[1]
    gn = _num_grad(f, th)
    assert np.abs(g - gn).max() <= 1e-7 * max(1.0, np.abs(gn).max())


def test_post_gradient_matches_central_differences(rng):
    n, b = 16, 5
    mb = T.dct2(n)[:b]
    db = T.dst7(n)[:b]
    wb = adjust.weights(n)[:b]
    q0 = adjust.procrustes(mb, db)
    phi = rng.uniform(-0.3, 0.3, b * (b - 1) // 2)
    f = lambda p: adjust.post_objective(p, q0, mb, db, wb, b)[0]
    g = adjust.post_objective(phi, q0, mb, db, wb, b)[1]
    gn = _num_grad(f, phi)
    assert np.abs(g - gn).max() <= 1e-7 * max(1.0, np.abs(gn).max())


def test_procrustes_closed_form_is_optimal_for_uniform_weights(rng):
    # orthogonal Procrustes: Q = U V^T is the global minimiser of ||Q M - D||_F
    n, b = 32, 8
    mb, db = T.dct2(n)[:b], T.dst7(n)[:b]
    q = adjust.procrustes(mb, db)
    assert np.abs(q.T @ q - np.eye(b)).max() < 1e-12
    best = np.sum((q @ mb - db) ** 2)
    for _ in range(200):
        z = rng.standard_normal((b, b)) * 0.05
        r = np.linalg.qr(np.eye(b) + z)[0]
        assert np.sum((r @ q @ mb - db) ** 2) >= best - 1e-12
    # the unweighted fit_post returns exactly this
    qf, _ = adjust.fit_post("C2", "S7", n, b, weighted=False)
    assert np.abs(qf - q).max() < 1e-14


def test_weighted_fit_not_worse_than_procrustes():
    n, b = 32, 8
    q0, j0 = adjust.fit_post("C2", "S7", n, b, weighted=False)
    q1, j1 = adjust.fit_post("C2", "S7", n, b, weighted=True)
    assert j1 <= j0 + 1e-12


def test_eq2_weights():
    w = adjust.weights(32)
    assert w[0] == 1.0
    # alpha = ln(100)/N: the weight falls by 100x over N rows
    assert abs(w[-1] * np.exp(-np.log(100) / 32) - 0.01) < 1e-12


def test_eq5_post_flip_is_chessboard(rng):
    # S (C DCT-2) R == (S C S) DCT-2 with C = blkdiag(Q, I)
    n, b = 16, 8
    q = np.linalg.qr(rng.standard_normal((b, b)))[0]
    c = adjust.post_matrix(n, q)
    s, r = T.signs(n), T.reversal(n)
    lhs = adjust.adjusted("C2", n, c=c, flip=True)
    rhs = (s @ c @ s) @ T.dct2(n)
    assert np.abs(lhs - rhs).max() < 1e-13
    assert np.abs(lhs - s @ c @ T.dct2(n) @ r).max() < 1e-13


def test_only_one_adjustment():
    with pytest.raises(ValueError):
        adjust.adjusted("C2", 8, a=np.eye(8), c=np.eye(8))


def test_round_half_away():
    x = np.array([0.5, -0.5, 1.5, -1.5, 2.4999, -2.5001, 0.0])
    assert adjust.round_half_away(x).tolist() == [1, -1, 2, -2, 2, -3, 0]


def test_frozen_params_consistent(params):
    # the frozen FP64 values are orthogonal and reproduce the recorded criterion,
    # and the integer versions are their rounding at scale 2^a
    for e in params.values():
        if e["kind"] == "band":
            a = np.asarray(e["a_f64"])
            assert np.abs(a - adjust.band_matrix(e["n"], e["layers"], np.asarray(e["theta"]))).max() < 1e-15
            m = a
            h = adjust.adjusted(e["base"], e["n"], a=a)
            ival = np.asarray(e["a_int"])
        else:
            m = np.asarray(e["q_f64"])
            h = adjust.adjusted(e["base"], e["n"], c=adjust.post_matrix(e["n"], m))
            ival = np.asarray(e["q_int"])
        assert np.abs(m.T @ m - np.eye(m.shape[0])).max() < 1e-12
        assert abs(adjust.criterion(h, T.matrix(e["target"], e["n"])) - e["criterion"]) < 1e-9
        assert (ival == adjust.round_half_away(m * (1 << e["a_prec"]))).all()


def test_dst3_band_approximates_dst7_low_frequencies(params):
    # section 2.2: the lowest-frequency basis functions are well approximated
    for n in (16, 32, 64):
        e = params[f"band_S3_S7_N{n}_K4"]
        assert min(e["low_freq_corr"][:4]) > 0.99
    e = params["post_C2_S7_N64_B16"]
    assert min(e["low_freq_corr"]) > 0.99
