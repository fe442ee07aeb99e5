"""Exact orthonormal trigonometric transforms in FP64 (test infrastructure).

Rows are basis vectors (k = frequency, n = sample); the forward transform of a
column vector x is y = T x.  The paper names the transforms and the relations
between them (section 2.1 and eq. 3) without writing the matrices out; the
normalisations below are the ones under which those relations hold exactly:

  DCT-2  T[k,n] = sqrt(2/N) e_k cos(pi k (2n+1) / (2N)),      e_0 = 1/sqrt2, else 1
  DCT-3  = DCT-2^T
  DST-2  T[k,n] = sqrt(2/N) d_k sin(pi (k+1)(2n+1) / (2N)),   d_{N-1} = 1/sqrt2, else 1
  DST-3  = DST-2^T
  DST-7  T[k,n] = sqrt(4/(2N+1)) sin(pi (2k+1)(n+1) / (2N+1))
  DCT-8  T[k,n] = sqrt(4/(2N+1)) cos(pi (2k+1)(2n+1) / (4N+2))

The other sine transforms, the "remaining DSTs" the design study of Fig. 1
targets (section 2, the sparsity-objective example), in their orthonormal
forms with the same orientation (DST-6 is the transpose of the DST-7 above,
as the DST-VI / DST-VII pair are):

  DST-1  T[k,n] = sqrt(2/(N+1)) sin(pi (k+1)(n+1) / (N+1))
  DST-4  T[k,n] = sqrt(2/N) sin(pi (2k+1)(2n+1) / (4N))
  DST-5  T[k,n] = 2/sqrt(2N+1) sin(2 pi (k+1)(n+1) / (2N+1))
  DST-6  T[k,n] = 2/sqrt(2N+1) sin(pi (k+1)(2n+1) / (2N+1))
  DST-8  T[k,n] = sqrt(4/(2N-1)) f_k f_n sin(pi (2k+1)(2n+1) / (4N-2)),  f_{N-1} = 1/sqrt2, else 1

  R[m,n] = 1 if m = N-1-n (reversal);  S = diag((-1)^m) (alternating signs).

Pins (tests/test_oracle_transforms.py): orthogonality; the section 2.1
relations DCT-3 = DCT-2^T, DST-2 = R DCT-2 S, DST-3 = S DCT-2^T R; eq. 3
DCT-8 = S DST-7 R; eq. 4 S DCT-2 = DCT-2 R; agreement with scipy.fft's
orthonormal DCT/DST types 2 and 3; DST-7 rows equal the eigenvectors of the
second-difference matrix tridiag(-1, 2, -1) with last diagonal entry 1
(a textbook characterisation); the recursive even/odd DCT-2 below equals the
dense product; DST-1 and DST-4 equal scipy.fft's orthonormal types 1 and 4;
DST-6 is the transpose of DST-7; DST-5 and DST-8 rows equal the eigenvectors
of the second-difference matrix with their boundary rows (DST-5: last diagonal
entry 3; DST-8: first diagonal 3 and the last off-diagonal pair -sqrt2, the
symmetric form of its half-sample boundary), with eigenvalues 2 - 2 cos w at
the closed-form frequencies, plus hand-evaluated N = 4 entries; every matrix
is orthogonal.
"""

from __future__ import annotations

import numpy as np

KINDS = ("C2", "C3", "S2", "S3", "S7", "C8")
OTHER_DSTS = ("S1", "S4", "S5", "S6", "S7", "S8")


def dct2(n: int) -> np.ndarray:
    k = np.arange(n)[:, None].astype(np.float64)
    i = np.arange(n)[None, :].astype(np.float64)
    t = np.sqrt(2.0 / n) * np.cos(np.pi * k * (2 * i + 1) / (2 * n))
    t[0, :] *= 1.0 / np.sqrt(2.0)
    return t


def dct3(n: int) -> np.ndarray:
    return dct2(n).T.copy()


def dst2(n: int) -> np.ndarray:
    k = np.arange(n)[:, None].astype(np.float64)
    i = np.arange(n)[None, :].astype(np.float64)
    t = np.sqrt(2.0 / n) * np.sin(np.pi * (k + 1) * (2 * i + 1) / (2 * n))
    t[n - 1, :] *= 1.0 / np.sqrt(2.0)
    return t


def dst3(n: int) -> np.ndarray:
    return dst2(n).T.copy()


def dst7(n: int) -> np.ndarray:
    k = np.arange(n)[:, None].astype(np.float64)
    i = np.arange(n)[None, :].astype(np.float64)
    return np.sqrt(4.0 / (2 * n + 1)) * np.sin(np.pi * (2 * k + 1) * (i + 1) / (2 * n + 1))


def dct8(n: int) -> np.ndarray:
    k = np.arange(n)[:, None].astype(np.float64)
    i = np.arange(n)[None, :].astype(np.float64)
    return np.sqrt(4.0 / (2 * n + 1)) * np.cos(np.pi * (2 * k + 1) * (2 * i + 1) / (4 * n + 2))


def _grid(n: int):
    return np.arange(n)[:, None].astype(np.float64), np.arange(n)[None, :].astype(np.float64)


def dst1(n: int) -> np.ndarray:
    k, i = _grid(n)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * (k + 1) * (i + 1) / (n + 1))


def dst4(n: int) -> np.ndarray:
    k, i = _grid(n)
    return np.sqrt(2.0 / n) * np.sin(np.pi * (2 * k + 1) * (2 * i + 1) / (4 * n))


def dst5(n: int) -> np.ndarray:
    k, i = _grid(n)
    return 2.0 / np.sqrt(2 * n + 1) * np.sin(2 * np.pi * (k + 1) * (i + 1) / (2 * n + 1))


def dst6(n: int) -> np.ndarray:
    k, i = _grid(n)
    return 2.0 / np.sqrt(2 * n + 1) * np.sin(np.pi * (k + 1) * (2 * i + 1) / (2 * n + 1))


def dst8(n: int) -> np.ndarray:
    k, i = _grid(n)
    t = np.sqrt(4.0 / (2 * n - 1)) * np.sin(np.pi * (2 * k + 1) * (2 * i + 1) / (4 * n - 2))
    t[n - 1, :] /= np.sqrt(2.0)
    t[:, n - 1] /= np.sqrt(2.0)
    return t


def reversal(n: int) -> np.ndarray:
    """R of section 2.1: R[m, n] = 1 iff m = N-1-n."""
    return np.eye(n)[::-1].copy()


def signs(n: int) -> np.ndarray:
    """S of section 2.1: diagonal with (-1)^m."""
    return np.diag((-1.0) ** np.arange(n))


def matrix(kind: str, n: int) -> np.ndarray:
    return {"C2": dct2, "C3": dct3, "S2": dst2, "S3": dst3, "S7": dst7, "C8": dct8, "S1": dst1, "S4": dst4,
            "S5": dst5, "S6": dst6, "S8": dst8}[kind](n)


def dct2_fast(x: np.ndarray) -> np.ndarray:
    """DCT-2 of the last axis by the even/odd (partial butterfly) recursion.

    With N = 2M, E[n] = x[n] + x[N-1-n] and O[n] = x[n] - x[N-1-n] (n < M):
    the even outputs are the M-point DCT-2 of E scaled by 1/sqrt2, and the odd
    outputs are O projected on the odd basis rows (a dense M x M product).
    Used only to pin that the butterfly decomposition the GPU relies on is the
    same linear map as the dense matrix (section 2.1: DCT-2 has fast
    algorithms).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    if n == 1:
        return x.copy()
    m = n // 2
    e = x[..., :m] + x[..., ::-1][..., :m]
    o = x[..., :m] - x[..., ::-1][..., :m]
    y = np.empty_like(x)
    y[..., 0::2] = dct2_fast(e) / np.sqrt(2.0)
    k = np.arange(1, n, 2)[:, None]
    i = np.arange(m)[None, :]
    odd_rows = np.sqrt(2.0 / n) * np.cos(np.pi * k * (2 * i + 1) / (2 * n))
    y[..., 1::2] = o @ odd_rows.T
    return y
