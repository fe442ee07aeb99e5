"""Pins of oracle.refit: finite differences, reductions to eq. 2, special cases."""

import numpy as np
import pytest

import synth
from oracle import adjust, refit
from oracle import transforms as T


def _fd(f, th, h=1e-6):
    g = np.zeros_like(th)
    for i in range(len(th)):
        e = np.zeros_like(th)
        e[i] = h
        g[i] = (f(th + e) - f(th - e)) / (2 * h)
    return g


@pytest.mark.parametrize("base", ["C2", "S3"])
def test_loss_gradient_matches_central_differences(base):
    x = synth.ar1_vectors(200, 32, 0.85, 0.99, 1.0, seed=4)
    th = np.random.Generator(np.random.PCG64(2)).uniform(-0.4, 0.4, 31)
    g = refit.grad(th, x, base=base)
    gn = _fd(lambda t: refit.loss(t, x, base=base), th)
    assert np.abs(g - gn).max() <= 1e-7 * max(1.0, np.abs(gn).max())


def test_lambda_zero_is_eq2_with_unit_weights_on_first_rows():
    x = synth.ar1_vectors(10, 32, 0.9, 0.9, 1.0, seed=1)
    th = np.random.Generator(np.random.PCG64(3)).uniform(-0.3, 0.3, 31)
    w = (np.arange(32) < 8).astype(np.float64)
    f, g = adjust.band_objective(th, T.dct2(32), T.dst7(32), 32, 2, w)
    assert abs(refit.loss(th, x, lam=0.0) - f) < 1e-12
    assert np.abs(refit.grad(th, x, lam=0.0) - g).max() < 1e-12


def test_energy_term_vanishes_on_first_basis_rows():
    # data spanned by the first 8 rows of H keeps all its energy there
    th = np.random.Generator(np.random.PCG64(5)).uniform(-0.3, 0.3, 31)
    h = T.dct2(32) @ adjust.band_matrix(32, 2, th)
    coef = np.random.Generator(np.random.PCG64(6)).standard_normal((50, 8))
    x = coef @ h[:8]
    _, energy, _ = refit.loss_terms(th, x)
    assert abs(energy) < 1e-12


def test_backward_is_adjoint_of_forward():
    rng = np.random.Generator(np.random.PCG64(7))
    x = rng.standard_normal((20, 32))
    gy = rng.standard_normal((20, 32))
    th = rng.uniform(-0.5, 0.5, 31)
    dx, dth = refit.backward(th, x, gy)
    # <gy, H dx'> == <H^T gy, dx'>  and the angle part by central differences
    v = rng.standard_normal((20, 32))
    assert abs(np.sum(gy * refit.forward(th, v)) - np.sum(dx * v)) < 1e-10
    gn = _fd(lambda t: float(np.sum(gy * refit.forward(t, x))), th)
    assert np.abs(dth - gn).max() <= 1e-7 * max(1.0, np.abs(gn).max())


def test_workload_vectors_shape_and_rho_range():
    x = synth.ar1_vectors(1000, 32, 0.85, 0.99, 1.0, seed=synth.SEED_BASE + 4)
    assert x.shape == (1000, 32)
    # a lag-1 correlation inside [0.85, 0.99] on average
    r = np.mean(x[:, 17:] * x[:, 16:-1]) / np.mean(x[:, 16:-1] ** 2)
    assert 0.85 < r < 0.99
