"""ORACLE (test infrastructure only): the objects of the ParaDiag method, each
from its own definition.

Section 2 (Algorithm 1) and Section 4 (Algorithm 3, alpha-circulant variant)
of Gander & Palitta, generalised with a mass matrix M: the all-at-once
equation is (M + tau K) U - M U Sigma_1^T = G, every shifted block becomes
P_i = (1 - pi_i) M + tau K and the capacitance matrix
J_ell = I + alpha^(1/ell) sum_i gamma_i P_i^{-1} M.

Nothing here chains the algorithm's steps: the spectrum of G, the blockwise
shifted solves, the alpha-circulant solution U_1 (by stepping, with no
Fourier transform), b (a time slice of U_1), x = J_ell^{-1} b and the
projection method of Section 3 are computed separately, so that the pins can
check the Sherman-Morrison-Woodbury identities that connect them.

Notation (paper): F is the ell x ell DFT matrix F_{jk} = omega^{(j-1)(k-1)},
omega = exp(-2 pi i / ell); pi = alpha^(1/ell) F C_1 e_1 are the eigenvalues
of the (alpha-)circulant, gamma = F^{-T} e_ell; D_alpha =
diag(1, alpha^(1/ell), ..., alpha^((ell-1)/ell)).  Arrays are time-major, so
the paper's "post-multiply by F^T" is an FFT along axis 0 here.

Every piece uses plain library primitives (numpy FFT, scipy sparse LU, dense
numpy solves); nothing is blocked or fused.
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


def galerkin_projection(cap, Msp, Ksp, tau, b, eps=1e-8, maxit=50, q=1):
    """Section 3: the projection method for J_ell x = b on a polynomial
    Krylov space, written from its definition.

    The space is K_m(A, b) with A = tau M^{-1} K (the paper's K_m(K, b) when
    M = I; a scalar multiple of the operator spans the same space).  An
    orthonormal basis V_m is built by Arnoldi with two Gram-Schmidt passes,
    and the iterate x_m = V_m y is fixed by the Galerkin condition
    V_m^T (J_ell x_m - b) = 0, i.e. (V_m^T J_ell V_m) y = ||b|| e_1, with
    J_ell applied to each basis vector through its definition (the sparse LU
    solves of ``Capacitance``).  The residual ||J_ell x_m - b|| is evaluated
    directly, every q-th dimension and at maxit, and the iteration stops
    once it is at most eps ||b||.

    The paper reaches the same projected matrix without applying J_ell to
    the basis, through the shifted Arnoldi relation (eq. compute_ym), and the
    same residual through eq. compute_resnorm; the pins compare those
    formulas with this direct evaluation.  Returns (x, m, residual norms at
    the checks)."""
    b = np.asarray(b, dtype=np.float64)
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros_like(b), 0, [0.0]
    Mlu = spla.splu(Msp.tocsc())
    basis = [b / beta]
    images = []                 # J_ell applied to each basis vector
    hist = []
    x = np.zeros_like(b)
    m = 0
    exhausted = False
    while m < maxit and not exhausted:
        m += 1
        images.append(cap.matvec(basis[m - 1]).real)
        # next basis vector: A v_m orthogonalised against the basis
        w = tau * Mlu.solve(Ksp @ basis[m - 1])
        size = float(np.linalg.norm(w))
        for _ in range(2):
            for v in basis:
                w = w - (v @ w) * v
        if float(np.linalg.norm(w)) <= 1e-13 * size:
            exhausted = True    # the space is invariant under A (m = nbar)
        else:
            basis.append(w / np.linalg.norm(w))
        if m % q == 0 or m == maxit or exhausted:
            Vm = np.array(basis[:m]).T
            Jm = Vm.T @ np.array(images).T
            rhs_m = np.zeros(m)
            rhs_m[0] = beta
            x = Vm @ np.linalg.solve(Jm, rhs_m)
            res = float(np.linalg.norm(cap.matvec(x).real - b))
            hist.append(res)
            if res <= eps * beta:
                break
    return x, m, hist


# --------------------------------------------------------------------------
# the pieces of the method, each from its own definition (Sections 2 and 4)
# --------------------------------------------------------------------------

def rhs_spectrum(Msp, tau, u0, F, alpha=1.0):
    """The right-hand side in Fourier variables, G D_alpha F^T (Section 2;
    Section 4 for the D_alpha scaling): row i is
    sum_t alpha^(t/ell) g_t omega^(t i), the un-normalised DFT along time of
    the scaled rows of G = M [u0 + tau f_1, tau f_2, ...]."""
    G = rhs(Msp, tau, u0, F)
    ell = G.shape[0]
    scale = (alpha ** (1.0 / ell)) ** np.arange(ell)
    return np.fft.fft(scale[:, None] * G, axis=0)


def shifted_solutions(cap, spec):
    """The block-diagonal operator of Section 2 applied blockwise: row i of
    the result is P_i^{-1} spec_i, P_i = (1 - pi_i) M + tau K."""
    out = np.empty(spec.shape, dtype=np.complex128)
    for i in range(spec.shape[0]):
        out[i] = cap.solve_shifted(i, spec[i])
    return out


def periodic_solution(Msp, Ksp, tau, u0, F, alpha=1.0, tol=1e-15):
    """U_1, the solution of the alpha-circulant all-at-once system
    (M + tau K) U - M U C_alpha^T = G (Sigma_1 with alpha in its corner;
    Section 2 for alpha = 1, Section 4), computed without any Fourier
    transform: backward-Euler stepping whose first step also sees
    alpha M u_ell.  Stepping from zero with the data G gives z, stepping
    the homogeneous problem ell times is Phi^ell with
    Phi = (M + tau K)^{-1} M, so u_ell solves (I - alpha Phi^ell) u_ell = z
    (by ``gmres``); one more stepping pass from u_0 := alpha u_ell gives
    every time slice."""
    G = rhs(Msp, tau, u0, F)
    ell, nbar = G.shape
    lu = spla.splu(sp.csc_matrix(Msp + tau * Ksp))

    def march(start, data):
        out = np.empty((ell, nbar))
        prev = start
        for j in range(ell):
            rhs_j = Msp @ prev
            if data is not None:
                rhs_j = rhs_j + data[j]
            out[j] = lu.solve(rhs_j)
            prev = out[j]
        return out

    z = march(np.zeros(nbar), G)[-1]
    op = lambda v: v - alpha * march(v, None)[-1]
    u_last, _, _ = gmres(op, z, tol=tol, maxit=min(nbar, 300))
    return march(alpha * np.real(u_last), G)


def capacitance_rhs(U1, alpha=1.0):
    """b = L F^{-T} e_ell (Section 2): since U_1 = L F^{-T} D_alpha^{-1},
    b = U_1 D_alpha e_ell = alpha^((ell-1)/ell) times the last time slice of
    the alpha-circulant solution."""
    ell = U1.shape[0]
    return (alpha ** (1.0 / ell)) ** (ell - 1) * U1[-1]


def capacitance_solution(cap, b, method="dense", tol=1e-14, maxit=200):
    """x = J_ell^{-1} b (eq. SMW_linearsystemII): a dense solve of the
    matrix J_ell formed column by column, or GMRES with J_ell applied
    through its definition."""
    if method == "dense":
        return np.linalg.solve(cap.dense(), b).real
    x, _, _ = gmres(lambda v: cap.matvec(v).real, np.asarray(b, dtype=np.float64), tol=tol,
                    maxit=maxit)
    return np.real(x)


def first_term_accepted(Msp, Ksp, tau, u0, F, U1, eps) -> bool:
    """Algorithm 3's test on the first term: U_1 is accepted when its
    residual in the original all-at-once system (with Sigma_1) is at most
    eps ||M U_1||_F.  The paper states the test for M = I against
    ||U_1||_F; with a mass matrix every residual row carries a factor M, so
    the bound uses ||M U_1||_F (the same test when M = I)."""
    R = rhs(Msp, tau, u0, F) - apply_allatonce(Msp, Ksp, tau, U1)
    MU1 = np.asarray((Msp @ U1.T).T)
    return bool(np.linalg.norm(R) <= eps * np.linalg.norm(MU1))


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
