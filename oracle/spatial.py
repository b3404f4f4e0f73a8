"""ORACLE (test infrastructure only): sparse spatial matrices.

The method takes the stiffness matrix K (and, for finite elements, the mass
matrix M) as its spatial input (Section 1).  1D problems give M and K as
tridiagonals; 2D problems give the 1D factor T and K = I (x) T + T (x) I with
M = I (Section 6.1, 2D heat equation)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def tridiag_sparse(t) -> sp.csr_matrix:
    lower, diag, upper = (np.asarray(a, dtype=np.float64) for a in t)
    n = diag.size
    return sp.diags([lower[1:], diag, upper[:-1]], [-1, 0, 1], shape=(n, n),
                    format="csr")


def spatial_matrices(M, K, dims: int):
    """Return (Msp, Ksp) as sparse nbar x nbar matrices."""
    T = tridiag_sparse(K)
    n = T.shape[0]
    if dims == 1:
        Msp = sp.identity(n, format="csr") if M is None else tridiag_sparse(M)
        return Msp, T
    if M is not None:
        raise ValueError("2D problems use M = I")
    I = sp.identity(n, format="csr")
    Ksp = (sp.kron(I, T) + sp.kron(T, I)).tocsr()
    return sp.identity(n * n, format="csr"), Ksp


def problem_matrices(p):
    """Sparse (M, K) of a ``workloads.HeatProblem``."""
    return spatial_matrices(p.M, p.K, p.dims)
