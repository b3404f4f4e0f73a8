"""ORACLE (test infrastructure only): the all-at-once backward-Euler system.

Section 1, all-at-once equation: (I + tau K) U - U Sigma_1^T =
[u0 + tau f_1, tau f_2, ..., tau f_ell], with Sigma_1 the ell x ell matrix
with ones on the first subdiagonal.  With a mass matrix M (finite elements,
nodal data) the equation reads

    (M + tau K) U - M U Sigma_1^T = G,   G = M [u0 + tau f_1, tau f_2, ...].

Arrays are time-major: U[j] is the paper's column j+1 (time t_{j+1}).
"""
from __future__ import annotations

import ctypes

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import _native


def rhs(Msp, tau: float, u0: np.ndarray, F: np.ndarray) -> np.ndarray:
    """G = M [u0 + tau f_1, tau f_2, ..., tau f_ell]  (rows = time)."""
    H = tau * np.asarray(F, dtype=np.float64)
    H[0] = H[0] + u0
    return np.asarray((Msp @ H.T).T)


def apply_allatonce(Msp, Ksp, tau: float, U: np.ndarray) -> np.ndarray:
    """(M + tau K) U - M U Sigma_1^T, i.e. row j: (M+tau K) u_j - M u_{j-1},
    with u_{-1} = 0 (u0 lives in G)."""
    A = (Msp + tau * Ksp)
    out = np.asarray((A @ U.T).T)
    out[1:] -= np.asarray((Msp @ U[:-1].T).T)
    return out


def residual(Msp, Ksp, tau, u0, F, U):
    """R = G - A(U) and ||R||_F / ||G||_F."""
    G = rhs(Msp, tau, u0, F)
    R = G - apply_allatonce(Msp, Ksp, tau, U)
    return R, float(np.linalg.norm(R) / np.linalg.norm(G))


def sigma1(ell: int) -> np.ndarray:
    """Sigma_1: zeros with ones on the first subdiagonal (Section 2)."""
    return np.eye(ell, k=-1)


def dense_matrix(Msp, Ksp, tau: float, ell: int) -> np.ndarray:
    """Kronecker form I_ell (x) (M + tau K) - Sigma_1 (x) M acting on
    vec(U) = [u_1; ...; u_ell]."""
    Md = Msp.toarray()
    Ad = Md + tau * Ksp.toarray()
    return np.kron(np.eye(ell), Ad) - np.kron(sigma1(ell), Md)


def solve_dense(Msp, Ksp, tau, u0, F) -> np.ndarray:
    """O2: dense LU solve of the all-at-once system (tiny sizes only)."""
    ell, nbar = F.shape
    G = rhs(Msp, tau, u0, F)
    A = dense_matrix(Msp, Ksp, tau, ell)
    return np.linalg.solve(A, G.reshape(-1)).reshape(ell, nbar)


def step_1d(M, K, tau, u0, F) -> np.ndarray:
    """O1 for 1D tridiagonal M, K: sequential stepping with Thomas (C code)."""
    ell, n = F.shape
    lib = _native.lib()
    c = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    ptr = lambda a: a.ctypes.data_as(dp) if a is not None else None
    Ml, Md, Mu = (c(a) for a in M) if M is not None else (None, None, None)
    Kl, Kd, Ku = (c(a) for a in K)
    u0c, Fc = c(u0), c(F)
    U = np.empty((ell, n), dtype=np.float64)
    rc = lib.pd_oracle_step_1d(n, ell, float(tau), ptr(Ml), ptr(Md), ptr(Mu),
                               ptr(Kl), ptr(Kd), ptr(Ku), ptr(u0c), ptr(Fc),
                               ptr(U))
    if rc != 0:
        raise RuntimeError("pd_oracle_step_1d failed with code %d" % rc)
    return U


def step_sparse(Msp, Ksp, tau, u0, F) -> np.ndarray:
    """O1 for any sparse M, K (used for 2D): factor M + tau K once with a
    sparse LU, then step (M + tau K) u_j = M (u_{j-1} + tau f_j)."""
    ell, nbar = F.shape
    lu = spla.splu(sp.csc_matrix(Msp + tau * Ksp))
    U = np.empty((ell, nbar))
    prev = np.asarray(u0, dtype=np.float64)
    for j in range(ell):
        U[j] = lu.solve(Msp @ (prev + tau * F[j]))
        prev = U[j]
    return U


def step(p) -> np.ndarray:
    """O1 for a ``workloads.HeatProblem``."""
    if p.dims == 1:
        return step_1d(p.M, p.K, p.tau, p.u0, p.F)
    from .spatial import problem_matrices
    Msp, Ksp = problem_matrices(p)
    return step_sparse(Msp, Ksp, p.tau, p.u0, p.F)


def rel_err(U, Uref) -> float:
    """Relative Frobenius error ||U - Uref||_F / ||Uref||_F."""
    return float(np.linalg.norm(U - Uref) / np.linalg.norm(Uref))
