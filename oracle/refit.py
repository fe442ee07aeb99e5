"""Refit objective of the differentiable path, FP64 (test infrastructure).

The adjusted transform H(theta) = B A(theta), with A(theta) the K-tap band of
Givens layers (section 2, "sequential sets of parallel Givens rotations";
layer convention in oracle.adjust), is refitted on residual vectors by
minimising

  L(theta) = sum_{i < P} ||h_i - d_i||^2
             + lam * (1 - sum_m sum_{i < P} y_{m,i}^2 / sum_m ||x_m||^2),

  y_m = H x_m,  d_i = rows of the exact DST-7,

i.e. eq. 2's row-weighted distance with unit weight on the first P = 8 rows
(the low-frequency basis functions the paper cares about, section 2.2) plus
an energy-compaction term on data (the fraction of energy outside the first P
coefficients).  The paper states no such combined objective; this reading
(lam = 1, P = 8) is a refit criterion built from its two stated goals.

Analytic gradient: with G = dL/dA =
    2 B^T Pm (B A - D)  -  (2 lam / E) B^T Pm B A S,
S = sum_m x_m x_m^T, E = sum_m ||x_m||^2, Pm = diag(i < P), the angle
gradient is oracle.adjust.band_grad(G).

Pins (tests/test_oracle_refit.py): central differences in FP64; lam = 0
reduces to eq. 2 with 0/1 row weights (oracle.adjust.band_objective); the
energy term is zero at theta where H keeps all energy in the first P rows
of a data set spanned by those rows.
"""

from __future__ import annotations

import numpy as np

from . import adjust
from . import transforms as T


def loss_terms(theta, x, base="C2", n=32, layers=2, p=8, lam=1.0):
    """(basis term, energy term, total) for vectors x[m, n]."""
    a = adjust.band_matrix(n, layers, theta)
    h = T.matrix(base, n) @ a
    d = T.dst7(n)
    basis = float(np.sum((h[:p] - d[:p]) ** 2))
    y = np.asarray(x, np.float64) @ h.T
    e = float(np.sum(np.asarray(x, np.float64) ** 2))
    energy = lam * (1.0 - float(np.sum(y[:, :p] ** 2)) / e)
    return basis, energy, basis + energy


def loss(theta, x, **kw):
    return loss_terms(theta, x, **kw)[2]


def grad(theta, x, base="C2", n=32, layers=2, p=8, lam=1.0):
    """dL/dtheta, analytic."""
    x = np.asarray(x, np.float64)
    a = adjust.band_matrix(n, layers, theta)
    b = T.matrix(base, n)
    d = T.dst7(n)
    pm = np.diag((np.arange(n) < p).astype(np.float64))
    s = x.T @ x
    e = float(np.trace(s))
    g = 2.0 * b.T @ pm @ (b @ a - d) - (2.0 * lam / e) * (b.T @ pm @ b @ a @ s)
    return adjust.band_grad(n, layers, theta, g)


def forward(theta, x, base="C2", n=32, layers=2):
    """y_m = B A(theta) x_m for x[m, n]."""
    h = T.matrix(base, n) @ adjust.band_matrix(n, layers, theta)
    return np.asarray(x, np.float64) @ h.T


def backward(theta, x, gy, base="C2", n=32, layers=2):
    """(dx, dtheta) of sum(gy * forward(theta, x)): dx = gy H, and the angle
    gradient through G = B^T gy^T x."""
    b = T.matrix(base, n)
    a = adjust.band_matrix(n, layers, theta)
    gy = np.asarray(gy, np.float64)
    x = np.asarray(x, np.float64)
    dx = gy @ (b @ a)
    g = b.T @ gy.T @ x
    return dx, adjust.band_grad(n, layers, theta, g)
