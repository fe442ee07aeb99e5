"""Orthogonal adjustments and adjusted transforms in FP64 (test infrastructure).

Eq. 1: H = C B A approximates the desired transform D, with A and C taken
from subsets of sparse orthogonal matrices, and only one of A or C different
from the identity (section 2.2, last paragraph).  The two subsets chosen for
DST-7 (section 2.2, list after eq. 3, and Fig. 2) are

  * a band matrix A applied before the base transform ("K-tap" band), and
  * a top-left B x B sub-block C = blkdiag(Q, I) applied after the DCT-2.

Orthogonality is obtained, as section 2 suggests, by factoring the adjustment
into sequential layers of parallel Givens rotations.  Reading used here (the
paper does not spell the factorisation out):

  * rotation on the adjacent pair (p, p+1) with angle t maps
        v_p   = cos t * u_p - sin t * u_{p+1}
        v_p+1 = sin t * u_p + cos t * u_{p+1};
  * layer l rotates the pairs (l mod 2 + 2j, l mod 2 + 2j + 1);
  * A(theta) = G_{L-1} ... G_1 G_0, which has at most K = 2L non-zeros per row
    (L = 2: a 4-tap band with N-1 angles, 31 at N = 32; L = 3: 6 taps);
  * Q in O(B) is written Q = Q0 G(phi), Q0 the orthogonal Procrustes solution
    and G(phi) a product of B(B-1)/2 Givens rotations (all pairs, row-major).

Eq. 2 weights row i of the error by exp(-alpha i), alpha = ln(10^2)/N.

The DCT-8 versions follow eq. 3 (T_C8 = S T_S7 R): the flipped transform of H
is S H R; for the post-adjustment after the DCT-2 this is (S C S) DCT-2 by
eq. 4 and eq. 5.

Pins (tests/test_oracle_adjust.py): A(theta) is orthogonal with at most K
non-zeros per row and the stated angle count; the eq. 2 gradient matches
central differences; for uniform weights the sub-block fit reaches the
closed-form orthogonal Procrustes optimum; flipping obeys eq. 5; theta = 0
gives the base transform.
"""

from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

from . import transforms as T


# ---------------------------------------------------------------------------
# Givens layers (band pre-adjustment)
# ---------------------------------------------------------------------------

def layer_pairs(n: int, layer: int) -> list:
    start = layer % 2
    return [(p, p + 1) for p in range(start, n - 1, 2)]


def n_angles(n: int, layers: int) -> int:
    return sum(len(layer_pairs(n, l)) for l in range(layers))


def givens_layer(n: int, layer: int, theta: np.ndarray) -> np.ndarray:
    g = np.eye(n)
    for (p, q), t in zip(layer_pairs(n, layer), theta):
        c, s = np.cos(t), np.sin(t)
        g[p, p], g[p, q], g[q, p], g[q, q] = c, -s, s, c
    return g


def split_angles(n: int, layers: int, theta: np.ndarray) -> list:
    out, o = [], 0
    for l in range(layers):
        m = len(layer_pairs(n, l))
        out.append(np.asarray(theta[o:o + m], dtype=np.float64))
        o += m
    return out


def band_matrix(n: int, layers: int, theta: np.ndarray) -> np.ndarray:
    """A(theta) = G_{L-1} ... G_0."""
    a = np.eye(n)
    for l, th in enumerate(split_angles(n, layers, theta)):
        a = givens_layer(n, l, th) @ a
    return a


def band_grad(n: int, layers: int, theta: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    """Gradient of f(A(theta)) given gbar = df/dA (an N x N matrix).

    df/dtheta_r = <G_{>l}^T gbar G_{<l}^T, dG_l/dtheta_r>, where dG_l/dtheta_r
    is zero outside the 2x2 block of the rotated pair and equals
    [[-sin, -cos], [cos, -sin]] there.
    """
    ths = split_angles(n, layers, theta)
    gs = [givens_layer(n, l, th) for l, th in enumerate(ths)]
    out = []
    for l, th in enumerate(ths):
        left = np.eye(n)
        for g in gs[l + 1:]:
            left = g @ left                    # G_{L-1} ... G_{l+1}
        right = np.eye(n)
        for g in gs[:l]:
            right = g @ right                  # G_{l-1} ... G_0
        m = left.T @ gbar @ right.T
        for (p, q), t in zip(layer_pairs(n, l), th):
            c, s = np.cos(t), np.sin(t)
            out.append(-s * m[p, p] - c * m[p, q] + c * m[q, p] - s * m[q, q])
    return np.asarray(out)


# ---------------------------------------------------------------------------
# Sub-block post-adjustment
# ---------------------------------------------------------------------------

def all_pairs(b: int) -> list:
    return [(p, q) for p in range(b) for q in range(p + 1, b)]


def rotation_product(b: int, phi: np.ndarray) -> np.ndarray:
    g = np.eye(b)
    for (p, q), t in zip(all_pairs(b), phi):
        r = np.eye(b)
        c, s = np.cos(t), np.sin(t)
        r[p, p], r[p, q], r[q, p], r[q, q] = c, -s, s, c
        g = r @ g
    return g


def rotation_product_grad(b: int, phi: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    rs = []
    for (p, q), t in zip(all_pairs(b), phi):
        r = np.eye(b)
        c, s = np.cos(t), np.sin(t)
        r[p, p], r[p, q], r[q, p], r[q, q] = c, -s, s, c
        rs.append(r)
    # prefix (right) products P_k = R_{k-1} ... R_0, suffix (left) products
    nr = len(rs)
    right = [np.eye(b)]
    for r in rs:
        right.append(r @ right[-1])
    left = [np.eye(b)] * (nr + 1)
    acc = np.eye(b)
    for k in range(nr - 1, -1, -1):
        left[k] = acc                             # R_{nr-1} ... R_{k+1}
        acc = acc @ rs[k]
    out = np.empty(nr)
    for k, ((p, q), t) in enumerate(zip(all_pairs(b), phi)):
        m = left[k].T @ gbar @ right[k].T
        c, s = np.cos(t), np.sin(t)
        out[k] = -s * m[p, p] - c * m[p, q] + c * m[q, p] - s * m[q, q]
    return out


def post_matrix(n: int, q: np.ndarray) -> np.ndarray:
    """C = blkdiag(Q, I_{N-B}) (Fig. 2b: only the top-left B x B block adjusts)."""
    b = q.shape[0]
    c = np.eye(n)
    c[:b, :b] = q
    return c


# ---------------------------------------------------------------------------
# Adjusted transforms (eq. 1) and their DCT-8 flips (eq. 3, eq. 5)
# ---------------------------------------------------------------------------

def adjusted(base: str, n: int, a: np.ndarray | None = None, c: np.ndarray | None = None,
             flip: bool = False) -> np.ndarray:
    """H = C B A, then S H R when ``flip`` (the DCT-8 version of a DST-7 design)."""
    if a is not None and c is not None:
        raise ValueError("only one of A or C is used at a time")
    h = T.matrix(base, n)
    if a is not None:
        h = h @ a
    if c is not None:
        h = c @ h
    if flip:
        h = T.signs(n) @ h @ T.reversal(n)
    return h


def weights(n: int) -> np.ndarray:
    """Row weights of eq. 2: exp(-alpha i), alpha = ln(10^2)/N."""
    alpha = np.log(100.0) / n
    return np.exp(-alpha * np.arange(n))


def criterion(h: np.ndarray, d: np.ndarray, w: np.ndarray | None = None) -> float:
    """Eq. 2: sum_i sum_j w_i (H_ij - D_ij)^2."""
    if w is None:
        w = weights(h.shape[0])
    return float(np.sum(w[:, None] * (h - d) ** 2))


def band_objective(theta, base_m, d, n, layers, w):
    a = band_matrix(n, layers, theta)
    err = base_m @ a - d
    f = float(np.sum(w[:, None] * err ** 2))
    gbar = 2.0 * base_m.T @ (w[:, None] * err)
    return f, band_grad(n, layers, theta, gbar)


def fit_band(base: str, target: str, n: int, taps: int, maxiter: int = 3000):
    """Minimise eq. 2 over the angles of a K-tap Givens band, from theta = 0."""
    layers = taps // 2
    base_m = T.matrix(base, n)
    d = T.matrix(target, n)
    w = weights(n)
    th0 = np.zeros(n_angles(n, layers))
    res = minimize(band_objective, th0, args=(base_m, d, n, layers, w), jac=True,
                   method="L-BFGS-B", options=dict(maxiter=maxiter, gtol=1e-12, ftol=1e-15))
    return res.x, float(res.fun)


def procrustes(m: np.ndarray, d: np.ndarray) -> np.ndarray:
    """argmin_{Q in O(B)} ||Q M - D||_F = U V^T with U S V^T = svd(D M^T)."""
    u, _, vt = np.linalg.svd(d @ m.T)
    return u @ vt


def post_objective(phi, q0, mb, db, wb, b):
    g = rotation_product(b, phi)
    q = q0 @ g
    err = q @ mb - db
    f = float(np.sum(wb[:, None] * err ** 2))
    gq = 2.0 * (wb[:, None] * err) @ mb.T            # df/dQ
    return f, rotation_product_grad(b, phi, q0.T @ gq)


def fit_post(base: str, target: str, n: int, b: int, maxiter: int = 3000, weighted: bool = True):
    """Fit the B x B sub-block after ``base`` (the DCT-2 in the paper).

    Rows i >= B of H are the base rows and do not depend on Q, so eq. 2
    reduces to the weighted problem over the first B rows.  Starts from the
    Procrustes solution (exact for uniform weights) and refines with L-BFGS
    over Givens angles.  Returns (Q, eq. 2 value of the full H).
    """
    base_m = T.matrix(base, n)
    d = T.matrix(target, n)
    w = weights(n)
    mb, db, wb = base_m[:b], d[:b], w[:b]
    q0 = procrustes(mb, db)
    if not weighted:
        q = q0
    else:
        phi0 = np.zeros(b * (b - 1) // 2)
        res = minimize(post_objective, phi0, args=(q0, mb, db, wb, b), jac=True,
                       method="L-BFGS-B", options=dict(maxiter=maxiter, gtol=1e-12, ftol=1e-15))
        q = q0 @ rotation_product(b, res.x)
    h = post_matrix(n, q) @ base_m
    return q, criterion(h, d, w)


def round_half_away(x: np.ndarray) -> np.ndarray:
    """Round to nearest, ties away from zero (sign-symmetric)."""
    x = np.asarray(x, dtype=np.float64)
    return (np.sign(x) * np.floor(np.abs(x) + 0.5)).astype(np.int64)


def band_support(a: np.ndarray, tol: float = 0.0) -> list:
    """Column indices of the non-zeros of each row (|a_ij| > tol)."""
    return [np.nonzero(np.abs(row) > tol)[0] for row in a]
