"""ORACLE (test infrastructure only): exact modal solution (O3).

For zero Dirichlet data on a uniform grid, the nodal sine vectors
s_k[i] = sin(k pi x_i), x_i = i h, are eigenvectors of every symmetric
Toeplitz tridiagonal matrix tridiag(d1, d0, d1) with eigenvalue
d0 + 2 d1 cos(k pi h) (Section 6.1 uses this for the 2D Laplacian, whose
eigenvalues are sums of the 1D ones).  When u0 and f are finite sine series,
the backward-Euler recurrence (M + tau K) u_j = M (u_{j-1} + tau f_j)
decouples into one scalar recurrence per mode,

    c_j = (c_{j-1} + tau fhat_j) / (1 + tau kappa / m),

which gives the discrete all-at-once solution to rounding error.  With f = 0
this is c_j = c_0 (1 + tau mu)^(-j).
"""
from __future__ import annotations

import numpy as np


def _toeplitz_symbol(t, k: int, h: float) -> float:
    lower, diag, upper = t
    n = diag.size
    d0 = float(diag[0])
    d1 = float(upper[0]) if n > 1 else 0.0
    if not (np.all(diag == d0) and np.all(upper[:-1] == d1)
            and np.all(lower[1:] == d1)):
        raise ValueError("modal oracle needs symmetric Toeplitz M and K")
    return d0 + 2.0 * d1 * np.cos(k * np.pi * h)


def _mode_series(tau, ell, m_k, kappa_k, c0, a, b):
    """Scalar backward-Euler recurrence for one mode, j = 1..ell."""
    out = np.empty(ell)
    c = c0
    ratio = 1.0 + tau * kappa_k / m_k
    for j in range(1, ell + 1):
        fhat = a * np.cos(b * j * tau) if a != 0.0 else 0.0
        c = (c + tau * fhat) / ratio
        out[j - 1] = c
    return out


def modal_solution(p) -> np.ndarray:
    """Exact discrete solution U [ell, nbar] of a ``workloads.HeatProblem``."""
    n, ell, tau, h = p.n, p.ell, p.tau, p.h
    x = np.arange(1, n + 1) * h
    if p.dims == 1:
        coeffs = {}
        for k, c in p.u0_modes.items():
            coeffs[k] = [c, 0.0, 0.0]
        for k in range(1, p.src_a.size + 1):
            coeffs.setdefault(k, [0.0, 0.0, 0.0])
            coeffs[k][1] = float(p.src_a[k - 1])
            coeffs[k][2] = float(p.src_b[k - 1])
        U = np.zeros((ell, n))
        for k, (c0, a, b) in sorted(coeffs.items()):
            m_k = 1.0 if p.M is None else _toeplitz_symbol(p.M, k, h)
            kap = _toeplitz_symbol(p.K, k, h)
            series = _mode_series(tau, ell, m_k, kap, c0, a, b)
            U += np.outer(series, np.sin(k * np.pi * x))
        return U
    # 2D, M = I, K = I (x) T + T (x) I, f = 0
    if p.src_a.size:
        raise ValueError("2D modal oracle supports f = 0 only")
    U = np.zeros((ell, n, n))
    for (k, m), c0 in p.u0_modes.items():
        kap = _toeplitz_symbol(p.K, k, h) + _toeplitz_symbol(p.K, m, h)
        series = _mode_series(tau, ell, 1.0, kap, c0, 0.0, 0.0)
        U += series[:, None, None] * np.outer(np.sin(m * np.pi * x),
                                              np.sin(k * np.pi * x))[None]
    return U.reshape(ell, n * n)


def final_slice(p) -> np.ndarray:
    """u_ell, the exact final time slice."""
    return modal_solution(p)[-1]


def modal_sample(p, t_idx, i_idx) -> np.ndarray:
    """U[t_idx[s], i_idx[s]] of the exact solution, evaluated point by point
    (for full-size problems where U itself is too large to form on the CPU)."""
    t_idx = np.asarray(t_idx)
    i_idx = np.asarray(i_idx)
    n, ell, tau, h = p.n, p.ell, p.tau, p.h
    out = np.zeros(t_idx.shape)
    if p.dims == 1:
        coeffs = {}
        for k, c in p.u0_modes.items():
            coeffs[k] = [c, 0.0, 0.0]
        for k in range(1, p.src_a.size + 1):
            coeffs.setdefault(k, [0.0, 0.0, 0.0])
            coeffs[k][1] = float(p.src_a[k - 1])
            coeffs[k][2] = float(p.src_b[k - 1])
        for k, (c0, a, b) in sorted(coeffs.items()):
            m_k = 1.0 if p.M is None else _toeplitz_symbol(p.M, k, h)
            kap = _toeplitz_symbol(p.K, k, h)
            series = _mode_series(tau, ell, m_k, kap, c0, a, b)
            out += series[t_idx] * np.sin(k * np.pi * (i_idx + 1) * h)
        return out
    y = i_idx // n
    x = i_idx % n
    for (k, m), c0 in p.u0_modes.items():
        kap = _toeplitz_symbol(p.K, k, h) + _toeplitz_symbol(p.K, m, h)
        series = _mode_series(tau, ell, 1.0, kap, c0, 0.0, 0.0)
        out += series[t_idx] * np.sin(m * np.pi * (y + 1) * h) * \
            np.sin(k * np.pi * (x + 1) * h)
    return out
