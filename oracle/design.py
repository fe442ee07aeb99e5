"""The adjustment design study of section 2 (Fig. 1), in FP64 (test infrastructure).

Section 2 obtains candidate adjustments without a prescribed sparsity pattern
by minimising, over all orthogonal matrices, the weighted approximation error
of eq. 2 plus a term that favours small entries (the unnumbered objective
printed after Fig. 2's caption, with C = I; the same with A = I for the
post-adjustment).  Fig. 1 shows the results for B in {DCT-2, DCT-3, DST-2,
DST-3} and D among the other DSTs.  Reading used here:

  objective     f(M) = lam sum_ij M_ij^2 / (0.05 + |M_ij|)
                       + sum_ij w_i (H_ij - D_ij)^2,    w_i = exp(-alpha i),
                alpha = ln(10^2) / N, lam = 1 as printed (lam = 0 is eq. 2)
  modes         pre-adjustment M = A, H = B M;  post-adjustment M = C, H = M B
  orthogonality M = G(theta) J with G = G_{N-1} ... G_1 G_0 a "brick wall" of
                N layers of parallel Givens rotations on adjacent pairs (layer
                l rotates the pairs starting at l mod 2; rotation convention
                as in oracle.adjust), N(N-1)/2 angles, which parametrises
                SO(N); J = diag(sigma, 1, ..., 1) with sigma the sign of
                det(target), target = B^T D (pre) or D B^T (post), so the
                exact adjustment is reachable
  optimiser     Adam (Kingma and Ba, 2015) with bias correction, a fixed step
                size and betas (0.9, 0.999), eps 1e-8: the paper names no
                optimiser for this study; a batch of independent restarts is
                what a GPU does well, and a first-order method per restart is
                the natural fit
  angle order   layer by layer, pairs in increasing order within a layer

Pins (tests/test_oracle_design.py): G is orthogonal, the identity at
theta = 0, the 2x2 rotation in closed form, and its Jacobian has full rank
N(N-1)/2 (it covers SO(N)); D = B at theta = 0 has zero error and sparsity
term N / 1.05; the analytic gradient matches central differences in both
modes and for both signs of sigma; Adam's first step moves every angle by
exactly the step size against the gradient's sign; with lam = 0 Adam reaches
the closed-form optimum M = target (eq. 2 without sparsity is solved exactly
by an orthogonal M).
"""

from __future__ import annotations

import numpy as np

SPARSE_EPS = 0.05


def n_angles(n: int) -> int:
    return n * (n - 1) // 2


def layer_pairs(n: int, layer: int):
    return list(range(layer % 2, n - 1, 2))


def weights(n: int) -> np.ndarray:
    return np.exp(-np.log(100.0) / n * np.arange(n))


def givens_net(theta: np.ndarray, n: int) -> np.ndarray:
    """G = G_{N-1} ... G_0 applied to the identity (columns are the vectors)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (n_angles(n),)
    v = np.eye(n)
    r = 0
    for layer in range(n):
        for p in layer_pairs(n, layer):
            c, s = np.cos(theta[r]), np.sin(theta[r])
            up, uq = v[p].copy(), v[p + 1].copy()
            v[p] = c * up - s * uq
            v[p + 1] = s * up + c * uq
            r += 1
    return v


def target(b: np.ndarray, d: np.ndarray, mode: str) -> np.ndarray:
    return b.T @ d if mode == "pre" else d @ b.T


def sigma_for(b: np.ndarray, d: np.ndarray, mode: str) -> float:
    return 1.0 if np.linalg.det(target(b, d, mode)) > 0 else -1.0


def adjustment(theta: np.ndarray, n: int, sigma: float) -> np.ndarray:
    m = givens_net(theta, n)
    m[:, 0] *= sigma
    return m


def objective(theta, b, d, mode: str, sigma: float, lam: float = 1.0):
    """(f, sparsity term, error term) at theta."""
    n = b.shape[0]
    m = adjustment(theta, n, sigma)
    h = b @ m if mode == "pre" else m @ b
    sp = float((m * m / (SPARSE_EPS + np.abs(m))).sum())
    err = float((weights(n)[:, None] * (h - d) ** 2).sum())
    return lam * sp + err, sp, err


def gradient(theta, b, d, mode: str, sigma: float, lam: float = 1.0) -> np.ndarray:
    """df/dtheta by the chain rule through M, then backwards through the layers."""
    n = b.shape[0]
    theta = np.asarray(theta, dtype=np.float64)
    m = adjustment(theta, n, sigma)
    h = b @ m if mode == "pre" else m @ b
    gh = 2.0 * weights(n)[:, None] * (h - d)
    a = np.abs(m)
    gm = lam * m * (2 * SPARSE_EPS + a) / (SPARSE_EPS + a) ** 2       # d/dM of M^2 / (eps + |M|)
    gm = gm + (b.T @ gh if mode == "pre" else gh @ b.T)
    g = gm.copy()
    g[:, 0] *= sigma                                                 # through M = G J
    v = givens_net(theta, n)                                         # V_N = G
    grad = np.zeros_like(theta)
    # angles of layer l occupy [start[l], start[l] + len(pairs))
    starts = np.cumsum([0] + [len(layer_pairs(n, l)) for l in range(n)])
    for layer in reversed(range(n)):
        for k, p in enumerate(layer_pairs(n, layer)):
            r = starts[layer] + k
            # outputs v' of this rotation are the current rows p, p+1
            grad[r] = float((-g[p] * v[p + 1] + g[p + 1] * v[p]).sum())
            c, s = np.cos(theta[r]), np.sin(theta[r])
            # step back: inputs = G^T outputs, and the adjoint likewise
            vp, vq = v[p].copy(), v[p + 1].copy()
            v[p], v[p + 1] = c * vp + s * vq, -s * vp + c * vq
            gp, gq = g[p].copy(), g[p + 1].copy()
            g[p], g[p + 1] = c * gp + s * gq, -s * gp + c * gq
    return grad


def adam(theta0, b, d, mode: str, sigma: float, lam: float, lr: float, steps: int,
         beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """`steps` Adam updates from theta0; returns the final angles."""
    theta = np.array(theta0, dtype=np.float64)
    mom = np.zeros_like(theta)
    vel = np.zeros_like(theta)
    for t in range(1, steps + 1):
        g = gradient(theta, b, d, mode, sigma, lam)
        mom = beta1 * mom + (1 - beta1) * g
        vel = beta2 * vel + (1 - beta2) * g * g
        mhat = mom / (1 - beta1 ** t)
        vhat = vel / (1 - beta2 ** t)
        theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta
