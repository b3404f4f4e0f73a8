"""ORACLE (test infrastructure only): the DST-I sine matrix.

S[k, i] = sqrt(2/(n+1)) sin((k+1)(i+1) pi / (n+1)) is symmetric and
orthogonal (S S = I); it diagonalises every symmetric Toeplitz tridiagonal
tridiag(d1, d0, d1) with eigenvalues d0 + 2 d1 cos((k+1) pi / (n+1)).  The 2D
heat example of Section 6.1 uses the closed-form eigenvalues of T that this
matrix realises."""
from __future__ import annotations

import numpy as np


def sine_matrix(n: int) -> np.ndarray:
    """The integer product (k+1)(i+1) is reduced modulo 2(n+1) before it is
    scaled by pi/(n+1), so every phase is exact to rounding: unreduced, the
    phases reach ~n^2 pi/(n+1) radians and lose ~1e-12 for n ~ 4096."""
    k = np.arange(1, n + 1, dtype=np.int64)
    r = np.outer(k, k) % (2 * (n + 1))
    return np.sqrt(2.0 / (n + 1)) * np.sin(r * np.pi / (n + 1))


def dst1(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """Orthonormal DST-I along ``axis`` by explicit matrix product."""
    x = np.moveaxis(np.asarray(x), axis, -1)
    S = sine_matrix(x.shape[-1])
    return np.moveaxis(x @ S.T, -1, axis)
