"""ORACLE (test infrastructure only): ParaDiag for backward Euler, step by step.

Follows Section 2 (Algorithm 1) and Section 4 (Algorithm 3, alpha-circulant
variant) of Gander & Palitta, generalised with a mass matrix M: the
all-at-once equation is (M + tau K) U - M U Sigma_1^T = G and every shifted
block becomes P_i = (1 - pi_i) M + tau K, the capacitance matrix
J_ell = I + alpha^(1/ell) sum_i gamma_i P_i^{-1} M.

Notation (paper): F is the ell x ell DFT matrix F_{jk} = omega^{(j-1)(k-1)},
omega = exp(-2 pi i / ell); pi = alpha^(1/ell) F C_1 e_1 are the eigenvalues
of the (alpha-)circulant, gamma = F^{-T} e_ell; D_alpha =
diag(1, alpha^(1/ell), ..., alpha^((ell-1)/ell)).  Arrays are time-major, so
the paper's "post-multiply by F^T" is an FFT along axis 0 here.

Every step uses plain library primitives (numpy FFT, scipy sparse LU, dense
numpy solves); nothing is blocked, fused or reordered.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .allatonce import apply_allatonce, rhs


# --------------------------------------------------------------------------
# circulant diagonalisation (Section 2; Appendix, proof of Theorem 1)
# --------------------------------------------------------------------------

def dft_matrix(ell: int) -> np.ndarray:
    """F_{jk} = omega^{(j-1)(k-1)}, omega = exp(-2 pi i / ell)."""
    j = np.arange(ell)
    return np.exp(-2j * np.pi * np.outer(j, j) / ell)


def circulant_c1(ell: int, alpha: float = 1.0) -> np.ndarray:
    """C_alpha: ones on the first subdiagonal and alpha in the top-right
    corner (Section 2 for alpha = 1, Section 4 for general alpha)."""
    C = np.eye(ell, k=-1)
    C[0, ell - 1] = alpha
    return C


def circulant_eigs(ell: int, alpha: float = 1.0):
    """pi_i = alpha^(1/ell) omega^(i-1) and gamma_i = omega^(i-1) / ell,
    i = 1..ell: the closed forms of alpha^(1/ell) F C_1 e_1 and F^{-T} e_ell
    (Appendix: gamma = (1/ell) conj(F) e_ell, whose entries are the
    powers omega^{-(ell-1)(i-1)} = omega^{i-1})."""
    k = np.arange(ell)
    w = np.exp(-2j * np.pi * k / ell)
    return alpha ** (1.0 / ell) * w, w / ell


def shifted_matrix(Msp, Ksp, tau, pi_i):
    """P_i = (1 - pi_i) M + tau K."""
    return ((1.0 - pi_i) * Msp + tau * Ksp).tocsc()


# --------------------------------------------------------------------------
# the capacitance system (Section 2, eq. SMW_linearsystemII; Section 4)
# --------------------------------------------------------------------------

class Capacitance:
    """J_ell = I + alpha^(1/ell) sum_i gamma_i P_i^{-1} M, applied through
    sparse LU factors of every P_i."""

    def __init__(self, Msp, Ksp, tau, ell, alpha=1.0):
        self.M = Msp
        self.pi, self.gamma = circulant_eigs(ell, alpha)
        self.weight = alpha ** (1.0 / ell)
        self.lu = [spla.splu(shifted_matrix(Msp, Ksp, tau, p)) for p in self.pi]

    def solve_shifted(self, i, rhs_vec):
        return self.lu[i].solve(np.asarray(rhs_vec, dtype=np.complex128))

    def matvec(self, v):
        Mv = self.M @ v
        acc = np.zeros(v.shape, dtype=np.complex128)
        for i, g in enumerate(self.gamma):
            acc += g * self.solve_shifted(i, Mv)
        out = v + self.weight * acc
        return out

    def dense(self):
        n = self.M.shape[0]
        Md = self.M.toarray()
        J = np.eye(n, dtype=np.complex128)
        for i, g in enumerate(self.gamma):
            J += self.weight * g * self.lu[i].solve(Md.astype(np.complex128))
        return J


def gmres(matvec, b, tol=1e-12, maxit=200):
    """Textbook GMRES (Saad, Iterative Methods, Alg. 6.9) from x0 = 0 with
    modified Gram-Schmidt; the small least-squares problem is solved with
    numpy's lstsq at every step.  Returns (x, iterations, residual norms)."""
    b = np.asarray(b)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0, [0.0]
    V = [b / beta]
    H = np.zeros((maxit + 1, maxit), dtype=np.result_type(b, np.float64))
    hist = [beta]
    y = np.zeros(0)
    m = 0
    for j in range(maxit):
        w = matvec(V[j])
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        e1 = np.zeros(j + 2, dtype=H.dtype)
        e1[0] = beta
        y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
        res = float(np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y))
        hist.append(res)
        m = j + 1
        if res <= tol * beta or H[j + 1, j] == 0.0:
            break
        V.append(w / H[j + 1, j])
    x = sum(y[i] * V[i] for i in range(m))
    return x, m, hist


def fom(cap, Msp, Ksp, tau, b, eps=1e-8, maxit=50, q=1):
    """Algorithm 2: the FOM-like projection of J_ell x = b onto a polynomial
    Krylov space, with the residual computed (and the small system solved)
    every q-th iteration.

    The space is K_m(A, b) with A = tau M^{-1} K, which is the paper's
    K_m(K, b) when M = I (a scalar multiple does not change the space).  With
    the Arnoldi relation A V_m = V_m T_m + t_{m+1,m} v_{m+1} e_m^T every
    shifted operator P_i^{-1} M = (lambda_i I + A)^{-1}, lambda_i = 1 - pi_i,
    satisfies the shift-invariant relation of Section 3 (tau, which the
    printed relation leaves off the t_{m+1,m} term, is inside A here), so
      S_i = (lambda_i I_m + T_m)^{-1},  h_i = P_i^{-1} M v_{m+1},
      (I + w sum_i gamma_i (I - t_{m+1,m} V_m^T h_i e_m^T) S_i) y = beta e_1,
      ||r|| = |t_{m+1,m}| w || (I - V_m V_m^T) sum_i gamma_i h_i e_m^T S_i y ||
    (eq. compute_ym and eq. compute_resnorm, with the alpha weight w of
    Section 4 and gamma_i in the residual as in eq. compute_resnorm).
    The loop runs at most maxit iterations.  Returns (x, m, residual norms at
    the checks)."""
    b = np.asarray(b, dtype=np.float64)
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros_like(b), 0, [0.0]
    Mlu = spla.splu(Msp.tocsc())
    V = [b / beta]
    T = np.zeros((maxit + 1, maxit))
    m = 0
    res = np.inf
    hist = []
    y = np.zeros(0)
    lam = 1.0 - cap.pi
    while res > eps * beta and m < maxit:
        m += 1
        w = tau * Mlu.solve(Ksp @ V[m - 1])
        for k in range(m):
            T[k, m - 1] = V[k] @ w
            w = w - T[k, m - 1] * V[k]
        T[m, m - 1] = np.linalg.norm(w)
        V.append(w / T[m, m - 1])
        if m % q == 0 or m == maxit:
            Tm = T[:m, :m]
            t = T[m, m - 1]
            Vm = np.array(V[:m]).T                     # nbar x m
            Mv = Msp @ V[m]
            Z = np.eye(m, dtype=np.complex128)
            S, H = [], []
            for i, g in enumerate(cap.gamma):
                Si = np.linalg.inv(lam[i] * np.eye(m) + Tm)
                hi = cap.solve_shifted(i, Mv)
                pi_ = Vm.T @ hi
                em = np.zeros(m); em[-1] = 1.0
                Z += cap.weight * g * (np.eye(m) - t * np.outer(pi_, em)) @ Si
                S.append(Si)
                H.append(hi)
            e1 = np.zeros(m); e1[0] = beta
            y = np.linalg.solve(Z, e1).real
            z = sum(g * H[i] * (S[i][-1] @ y) for i, g in enumerate(cap.gamma))
            rho = z - Vm @ (Vm.T @ z)
            res = abs(t) * cap.weight * float(np.linalg.norm(rho))
            hist.append(res)
    x = np.array(V[:m]).T @ y
    return x, m, hist


# --------------------------------------------------------------------------
# Algorithm 1 / Algorithm 3
# --------------------------------------------------------------------------

def paradiag(Msp, Ksp, tau, u0, F, alpha=1.0, capacitance="dense",
             tol=1e-13, maxit=200, early_exit_eps=None, q=1):
    """ParaDiag with backward Euler.  Returns a dict with the intermediates
    of the method (pi, gamma, Ghat, L, U1, b, x, W) and the solution U.

    capacitance = "dense" forms J_ell explicitly and solves it with LU;
    "gmres" applies J_ell matrix-free and solves with ``gmres``; "fom" runs
    Algorithm 2 (``fom``, residual checks every ``q`` iterations).

    early_exit_eps: Algorithm 3's test on the first term -- if the residual
    of U_1 in the original all-at-once system (with Sigma_1, not C_alpha) is
    at most eps * ||M U_1||_F, U = U_1 and the capacitance solve and the
    second parfor are skipped (early_exit = True in the result).  The paper
    states the test for M = I against ||U_1||_F; with a mass matrix every
    row of the residual carries a factor M, so it is measured against
    ||M U_1||_F (the same test when M = I)."""
    ell, nbar = F.shape
    pi, gamma = circulant_eigs(ell, alpha)
    weight = alpha ** (1.0 / ell)
    Dalpha = weight ** np.arange(ell)
    G = rhs(Msp, tau, u0, F)
    # [u0 + tau f_1, ..., tau f_ell] D_alpha F^T  (with M applied: G)
    Ghat = np.fft.fft(Dalpha[:, None] * G, axis=0)
    cap = Capacitance(Msp, Ksp, tau, ell, alpha)
    # first parfor: L e_i = P_i^{-1} Ghat e_i
    L = np.empty((ell, nbar), dtype=np.complex128)
    for i in range(ell):
        L[i] = cap.solve_shifted(i, Ghat[i])
    # U_1 = L F^{-T} D_alpha^{-1}
    U1 = np.fft.ifft(L, axis=0) / Dalpha[:, None]
    if early_exit_eps is not None:
        R = rhs(Msp, tau, u0, F) - apply_allatonce(Msp, Ksp, tau, U1.real)
        MU1 = np.asarray((Msp @ U1.real.T).T)
        if np.linalg.norm(R) <= early_exit_eps * np.linalg.norm(MU1):
            return dict(pi=pi, gamma=gamma, G=G, Ghat=Ghat, L=L, U1=U1, b=None,
                        x=None, W=None, U=U1.real.copy(), gmres_iters=0,
                        early_exit=True)
    # b = L F^{-T} e_ell = sum_i gamma_i L e_i
    b = (gamma[:, None] * L).sum(axis=0)
    if capacitance == "dense":
        x = np.linalg.solve(cap.dense(), b)
        its = 0
    elif capacitance == "fom":
        x, its, _ = fom(cap, Msp, Ksp, tau, b.real, eps=tol, maxit=maxit, q=q)
    else:
        x, its, _ = gmres(cap.matvec, b, tol=tol, maxit=maxit)
    # second parfor: W e_i = P_i^{-1} M x
    Mx = Msp @ x
    W = np.empty((ell, nbar), dtype=np.complex128)
    for i in range(ell):
        W[i] = cap.solve_shifted(i, Mx)
    # U = U_1 - alpha^(1/ell) W F^{-T} D_alpha^{-1}
    U = U1 - weight * np.fft.ifft(W, axis=0) / Dalpha[:, None]
    return dict(pi=pi, gamma=gamma, G=G, Ghat=Ghat, L=L, U1=U1, b=b, x=x,
                W=W, U=U, gmres_iters=its, early_exit=False)


def smw_dense(Msp, Ksp, tau, u0, F, alpha=1.0) -> np.ndarray:
    """O4: the Sherman-Morrison-Woodbury formula of Section 2 (eq. SMW_U;
    Section 4, eq. SMW_U_alpha) evaluated literally with dense Kronecker
    matrices.  Tiny sizes only."""
    ell, nbar = F.shape
    Md = Msp.toarray()
    Kd = Ksp.toarray()
    Fm = dft_matrix(ell)
    Finv = np.linalg.inv(Fm)
    pi, _ = circulant_eigs(ell, alpha)
    Pi = np.diag(pi)
    weight = alpha ** (1.0 / ell)
    Dalpha = np.diag(weight ** np.arange(ell))
    e1 = np.zeros(ell); e1[0] = 1.0
    el = np.zeros(ell); el[-1] = 1.0
    I_n = np.eye(nbar)
    # P := I_ell (x) (M + tau K) - Pi (x) M  (block diagonal)
    P = np.kron(np.eye(ell), Md + tau * Kd) - np.kron(Pi, Md)
    # low-rank factors: Mcal = F e_1 (x) M, Ncal = F^{-T} e_ell (x) I
    Mcal = np.kron((Fm @ e1)[:, None], Md)
    Ncal = np.kron((Finv.T @ el)[:, None], I_n)
    G = rhs(Msp, tau, u0, F)            # rows = time; paper's G = G_rows^T
    Gp = G.T                            # nbar x ell, columns = time
    ghat = (Gp @ Dalpha @ Fm.T).T.reshape(-1)   # vec(G D_alpha F^T)
    Pinv_g = np.linalg.solve(P, ghat)
    Pinv_M = np.linalg.solve(P, Mcal)
    cap = np.eye(nbar) + weight * (Ncal.T @ Pinv_M)
    vec_Ut = Pinv_g - weight * Pinv_M @ np.linalg.solve(cap, Ncal.T @ Pinv_g)
    Ut = vec_Ut.reshape(ell, nbar).T    # nbar x ell
    Up = Ut @ np.linalg.inv(Fm.T) @ np.linalg.inv(Dalpha)
    return Up.T                         # back to time-major


def theorem1_bound(tau, lam_min_K) -> float:
    """Theorem 1: kappa(J_ell) <= 1 + 1 / (tau lambda_min(K))."""
    return 1.0 + 1.0 / (tau * lam_min_K)


def lambda_min_2d_laplacian(n: int) -> float:
    """Section 6.1: lambda_min(K) = (8/h^2) sin(pi / (2(n+1)))^2 for the
    5-point Laplacian on an n x n interior grid, h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    return 8.0 / h**2 * np.sin(np.pi / (2 * (n + 1)))**2


def j_extreme_eigs(tau, ell, lam_min_K, lam_max_K, alpha=1.0):
    """Section 6.1: lambda_min(J) = 1 + sum_i gamma_i / (1 - pi_i +
    tau lambda_max(K)) and lambda_max(J) likewise with lambda_min(K)
    (M = I)."""
    pi, gamma = circulant_eigs(ell, alpha)
    w = alpha ** (1.0 / ell)
    lo = 1.0 + w * np.sum(gamma / (1.0 - pi + tau * lam_max_K))
    hi = 1.0 + w * np.sum(gamma / (1.0 - pi + tau * lam_min_K))
    return lo, hi
