"""Pins of the oracle's adjustment design study (section 2, Fig. 1)."""

import math

import numpy as np
import pytest

from oracle import design as Dz
from oracle import transforms as T


def test_network_orthogonal_identity_and_angle_count():
    rng = np.random.default_rng(1)
    for n in (2, 3, 4, 8, 16):
        assert Dz.n_angles(n) == sum(len(Dz.layer_pairs(n, l)) for l in range(n))
        assert np.allclose(Dz.givens_net(np.zeros(Dz.n_angles(n)), n), np.eye(n))
        g = Dz.givens_net(rng.uniform(-3, 3, Dz.n_angles(n)), n)
        assert np.abs(g.T @ g - np.eye(n)).max() < 1e-13
        assert np.linalg.det(g) == pytest.approx(1.0)


def test_two_point_rotation_closed_form():
    t = 0.3
    g = Dz.givens_net(np.array([t]), 2)
    assert np.allclose(g, [[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
    # objective by hand: B = I, D = I, pre, lam = 1: error (g - I)^2 with w = (1, 100^(-1/2))
    b = np.eye(2)
    f, sp, err = Dz.objective(np.array([t]), b, b, "pre", 1.0)
    c, s = math.cos(t), math.sin(t)
    assert sp == pytest.approx(2 * c * c / (0.05 + c) + 2 * s * s / (0.05 + s))
    assert err == pytest.approx((c - 1) ** 2 + s * s + 0.1 * (s * s + (c - 1) ** 2))
    assert f == pytest.approx(sp + err)


@pytest.mark.parametrize("n", [4, 5, 6])
def test_network_covers_so_n(n):
    """Full-rank Jacobian of theta -> G: the N(N-1)/2 angles reach every
    direction of SO(N) at a generic point."""
    rng = np.random.default_rng(n)
    th = rng.uniform(-1, 1, Dz.n_angles(n))
    h = 1e-6
    jac = np.stack([(Dz.givens_net(th + h * e, n) - Dz.givens_net(th - h * e, n)).ravel() / (2 * h)
                    for e in np.eye(len(th))], axis=1)
    assert np.linalg.matrix_rank(jac, tol=1e-6) == Dz.n_angles(n)


def test_base_equal_to_target_is_exact_at_zero():
    for kind in ("C2", "S3", "S7"):
        b = T.matrix(kind, 8)
        f, sp, err = Dz.objective(np.zeros(Dz.n_angles(8)), b, b, "pre", 1.0)
        assert err == 0.0 and sp == pytest.approx(8 / 1.05)


@pytest.mark.parametrize("mode", ["pre", "post"])
@pytest.mark.parametrize("sigma", [1.0, -1.0])
@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_gradient_matches_central_differences(mode, sigma, lam):
    n = 6
    rng = np.random.default_rng(7)
    b, d = T.matrix("S3", n), T.matrix("S7", n)
    th = rng.uniform(-0.8, 0.8, Dz.n_angles(n))
    g = Dz.gradient(th, b, d, mode, sigma, lam)
    h = 1e-6
    fd = np.array([(Dz.objective(th + h * e, b, d, mode, sigma, lam)[0] -
                    Dz.objective(th - h * e, b, d, mode, sigma, lam)[0]) / (2 * h) for e in np.eye(len(th))])
    assert np.abs(g - fd).max() < 1e-6 * max(1.0, np.abs(fd).max())


def test_adam_first_step_is_signed_step_size():
    n = 5
    rng = np.random.default_rng(3)
    b, d = T.matrix("C2", n), T.matrix("S4", n)
    th0 = rng.uniform(-0.5, 0.5, Dz.n_angles(n))
    g = Dz.gradient(th0, b, d, "pre", 1.0)
    th1 = Dz.adam(th0, b, d, "pre", 1.0, 1.0, 0.01, 1)
    assert np.allclose(th1 - th0, -0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), atol=1e-15)


@pytest.mark.parametrize("mode", ["pre", "post"])
def test_without_sparsity_adam_reaches_the_exact_adjustment(mode):
    """lam = 0 is eq. 2 over all of O(N): M = target is the exact solution."""
    n = 4
    b, d = T.matrix("S3", n), T.matrix("S7", n)
    sg = Dz.sigma_for(b, d, mode)
    th = Dz.adam(np.zeros(Dz.n_angles(n)), b, d, mode, sg, 0.0, 0.02, 3000)
    f, _, err = Dz.objective(th, b, d, mode, sg, 0.0)
    assert err < 1e-6
    assert np.abs(Dz.adjustment(th, n, sg) - Dz.target(b, d, mode)).max() < 2e-3
