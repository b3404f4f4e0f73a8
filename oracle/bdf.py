"""ORACLE (test infrastructure only): backward differentiation formulas of
order s <= 6 in the all-at-once setting of Section 5, with a mass matrix.

    (M + tau beta K) U - M U Sigma_s^T = G_s,
    row t of G_s (time t+1):  M (sum_{j=t+1}^{s} alpha_j u_{t+1-j} + tau beta f_{t+1}),

with s initial values u_{1-s}, ..., u_0 (passed as U0[0..s-1] in that
order) and Sigma_s lower-triangular Toeplitz with alpha_j on its j-th
subdiagonal.  Sigma_s = C_s - [e_1..e_s] A_s [e_{ell-s+1}..e_ell]^T with C_s
the circulant whose first column carries alpha_1..alpha_s in rows 2..s+1 and
A_s the s x s upper-triangular block (A_s)_{r,c} = alpha_{s-c+r}, c >= r
(0-based), the wrapped-around entries of C_s.

ParaDiag for BDF (Section 5): P_i = (1 - pi_i) M + tau beta K with
pi = F C_s e_1, theta^(h) = F e_h, gamma^(k) = F^{-T} [e_{ell-s+1}..e_ell]
A_s^T e_k, the s x s block capacitance matrix J^(s) with blocks
delta_{kh} I + sum_i gamma_i^(k) theta_i^(h) P_i^{-1} M, b^(s)_k =
sum_i gamma_i^(k) P_i^{-1} Ghat_i, and U = (L - W) F^{-T} with
W e_i = P_i^{-1} M sum_h theta_i^(h) x_h.  The transposes on A_s follow from
N = F^{-T}[e_{ell-s+1}..e_ell] A_s^T (the printed definition of gamma^(i)
uses A_s e_i; the transposed form is the one that reproduces the dense
solution, see the pins).  The capacitance system is solved densely or by
the block Galerkin method of the Proposition (``block_galerkin``), whose
block matrices are (s sm) x (s sm) with s x s blocks of size sm (the
printed R^{ms x ms} is read that way).  Arrays are time-major; FFTs run
along axis 0."""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np
import scipy.sparse.linalg as spla

from .modal import _toeplitz_symbol

# Table of BDF coefficients (Section 5): beta and alpha_1..alpha_s, signs as
# printed (u_n - sum_j alpha_j u_{n-j} = tau beta f_n).
BDF = {
    1: (Fr(1), [Fr(1)]),
    2: (Fr(2, 3), [Fr(4, 3), Fr(-1, 3)]),
    3: (Fr(6, 11), [Fr(18, 11), Fr(-9, 11), Fr(2, 11)]),
    4: (Fr(12, 25), [Fr(48, 25), Fr(-36, 25), Fr(16, 25), Fr(-3, 25)]),
    5: (Fr(60, 137), [Fr(300, 137), Fr(-300, 137), Fr(200, 137), Fr(-75, 137), Fr(12, 137)]),
    6: (Fr(60, 147), [Fr(360, 147), Fr(-450, 147), Fr(400, 147), Fr(-225, 147), Fr(72, 147),
                      Fr(-10, 147)]),
}


def coefficients(s: int):
    beta, alpha = BDF[s]
    return float(beta), np.array([float(a) for a in alpha])


def rhs_bdf(Msp, tau, s, U0, F):
    beta, alpha = coefficients(s)
    H = tau * beta * np.asarray(F, dtype=np.float64)
    for t in range(min(s, H.shape[0])):
        for j in range(t + 1, s + 1):
            H[t] += alpha[j - 1] * U0[s - 1 - (j - t - 1)]   # u_{t+1-j}
    return np.asarray((Msp @ H.T).T)


def apply_bdf(Msp, Ksp, tau, s, U):
    """(M + tau beta K) U - M U Sigma_s^T: row t is (M + tau beta K) u_t -
    M sum_j alpha_j u_{t-j} (terms with t - j < 0 are zero)."""
    beta, alpha = coefficients(s)
    out = np.asarray(((Msp + tau * beta * Ksp) @ U.T).T)
    for j in range(1, s + 1):
        out[j:] -= alpha[j - 1] * np.asarray((Msp @ U[:-j].T).T)
    return out


def sigma_s(ell, s):
    _, alpha = coefficients(s)
    S = np.zeros((ell, ell))
    for j in range(1, s + 1):
        S += alpha[j - 1] * np.eye(ell, k=-j)
    return S


def circulant_cs(ell, s):
    _, alpha = coefficients(s)
    c = np.zeros(ell)
    c[1:s + 1] = alpha
    return np.array([np.roll(c, k) for k in range(ell)]).T   # columns are shifts


def alpha_block(s):
    _, alpha = coefficients(s)
    A = np.zeros((s, s))
    for r in range(s):
        for c in range(r, s):
            A[r, c] = alpha[s - c + r - 1]
    return A


def step_bdf(Msp, Ksp, tau, s, U0, F):
    """Sequential BDF stepping (sparse LU of M + tau beta K)."""
    beta, alpha = coefficients(s)
    ell = F.shape[0]
    lu = spla.splu((Msp + tau * beta * Ksp).tocsc())
    hist = [np.asarray(u, dtype=np.float64) for u in U0]     # u_{1-s}..u_0
    out = np.empty((ell, F.shape[1]))
    for t in range(ell):
        acc = tau * beta * F[t]
        for j in range(1, s + 1):
            acc = acc + alpha[j - 1] * hist[-j]
        out[t] = lu.solve(Msp @ acc)
        hist.append(out[t])
    return out


def solve_dense_bdf(Msp, Ksp, tau, s, U0, F):
    beta, _ = coefficients(s)
    ell, nbar = F.shape
    Md = Msp.toarray()
    A = np.kron(np.eye(ell), Md + tau * beta * Ksp.toarray()) - np.kron(sigma_s(ell, s), Md)
    return np.linalg.solve(A, rhs_bdf(Msp, tau, s, U0, F).reshape(-1)).reshape(ell, nbar)


def _pieces(Msp, Ksp, tau, s, U0, F, gamma_transposed=True):
    """pi, theta^(h), gamma^(k), the LU of every P_i, L = P^{-1} Ghat and
    b^(s) (Section 5)."""
    beta, alpha = coefficients(s)
    ell, nbar = F.shape
    c = np.zeros(ell)
    c[1:s + 1] = alpha
    pi = np.fft.fft(c)                                   # F C_s e_1
    theta = [np.fft.fft(np.eye(ell)[h]) for h in range(s)]   # F e_h
    A = alpha_block(s)
    gamma = []
    for k in range(s):
        v = np.zeros(ell)
        v[ell - s:] = A[k, :] if gamma_transposed else A[:, k]
        gamma.append(np.fft.ifft(v))                     # F^{-T} = F^{-1}
    lus = [spla.splu(((1.0 - p) * Msp + tau * beta * Ksp).tocsc()) for p in pi]
    G = rhs_bdf(Msp, tau, s, U0, F)
    Ghat = np.fft.fft(G, axis=0)
    L = np.array([lus[i].solve(Ghat[i].astype(np.complex128)) for i in range(ell)])
    b = np.concatenate([(gamma[k][:, None] * L).sum(axis=0) for k in range(s)]).real
    return dict(pi=pi, theta=theta, gamma=gamma, lus=lus, L=L, b=b, beta=beta)


def paradiag_bdf(Msp, Ksp, tau, s, U0, F, gamma_transposed=True, capacitance="dense",
                 eps=1e-12, maxit=40):
    """ParaDiag for BDF-s following Section 5.  capacitance: "dense" solves
    the s*nbar capacitance system by dense LU (tiny sizes), "galerkin" by
    the block Galerkin method of the Proposition (``block_galerkin``)."""
    ell, nbar = F.shape
    P = _pieces(Msp, Ksp, tau, s, U0, F, gamma_transposed)
    pi, theta, gamma, lus, L, b = (P[k] for k in ("pi", "theta", "gamma", "lus", "L", "b"))
    Md = Msp.toarray().astype(np.complex128)
    PM = [lus[i].solve(Md) for i in range(ell)]
    J = np.eye(s * nbar, dtype=np.complex128)
    for k in range(s):
        for h in range(s):
            blk = sum(gamma[k][i] * theta[h][i] * PM[i] for i in range(ell))
            J[k * nbar:(k + 1) * nbar, h * nbar:(h + 1) * nbar] += blk
    extra = {}
    if capacitance == "galerkin":
        x, m, hist = block_galerkin(Msp, Ksp, tau, s, P, eps=eps, maxit=maxit)
        x = x.reshape(s, nbar)
        extra = dict(steps=m, history=hist)
    else:
        x = np.linalg.solve(J, b).real.reshape(s, nbar)
    W = np.array([lus[i].solve((Msp @ sum(theta[h][i] * x[h] for h in range(s)))
                               .astype(np.complex128)) for i in range(ell)])
    U = np.fft.ifft(L - W, axis=0).real
    U1 = np.fft.ifft(L, axis=0).real
    return dict(U=U, U1=U1, b=b, x=x, pi=pi, J=J.real, **extra)


def block_galerkin(Msp, Ksp, tau, s, pieces, eps=1e-12, maxit=40):
    """The block Galerkin method of Section 5 (Proposition) for
    J^(s) x = b^(s): block Arnoldi on A with the starting block
    B^(s) = [b_1 .. b_s] = V_1 beta (QR), x_k = V_m y_k, y from
    (I + T_m) y = (e_1 (x) I_s) beta with the (k, h) blocks
    sum_i gamma_i^(k) theta_i^(h) (S_i - V_m^T H_i t_{m+1,m} E_m^T S_i),
    S_i = ((1 - pi_i) I + T_m)^{-1}, H_i = P_i^{-1} M V_{m+1}, and the
    residual norm ||(I - I_s (x) V_m V_m^T) S_m y|| of the Proposition.
    With a mass matrix the Krylov operator is A = tau beta M^{-1} K
    (P_i^{-1} M = ((1 - pi_i) I + A)^{-1}; for M = I the paper's tau beta K
    with tau beta taken into T_m).  Returns (x, m, residual history)."""
    pi, theta, gamma, lus, b, beta = (pieces[k] for k in
                                      ("pi", "theta", "gamma", "lus", "b", "beta"))
    ell = len(pi)
    nbar = b.size // s
    Mlu = spla.splu(Msp.tocsc())

    def apply_A(W):
        return Mlu.solve(tau * beta * np.asarray(Ksp @ W))

    B = b.reshape(s, nbar).T                     # column k = b_k
    V1, bet = np.linalg.qr(B)
    Vs = [V1]
    T = np.zeros((s * (maxit + 1), s * maxit))
    coef = [[gamma[k] * theta[h] for h in range(s)] for k in range(s)]
    nb = np.linalg.norm(b)
    hist = []
    x = np.zeros(s * nbar)
    for m in range(1, maxit + 1):
        W = apply_A(Vs[-1])
        col = slice((m - 1) * s, m * s)
        for _ in range(2):                        # block classical Gram-Schmidt, twice
            for j, Vj in enumerate(Vs):
                h = Vj.T @ W
                T[j * s:(j + 1) * s, col] += h
                W = W - Vj @ h
        Q, R = np.linalg.qr(W)
        T[m * s:(m + 1) * s, col] = R
        Vm = np.hstack(Vs)
        Tm = T[:s * m, :s * m]
        sm = s * m
        H = [lus[i].solve(np.asarray(Msp @ Q).astype(np.complex128)) for i in range(ell)]
        S = [np.linalg.inv((1.0 - pi[i]) * np.eye(sm) + Tm) for i in range(ell)]
        ES = [R @ Si[-s:, :] for Si in S]          # t_{m+1,m} E_m^T S_i
        Tbig = np.eye(s * sm, dtype=np.complex128)
        Sbig = [[None] * s for _ in range(s)]
        for k in range(s):
            for h in range(s):
                Ssum = sum(coef[k][h][i] * (H[i] @ ES[i]) for i in range(ell))
                Sbig[k][h] = Ssum                   # nbar x sm
                Tsum = sum(coef[k][h][i] * S[i] for i in range(ell)) - Vm.T @ Ssum
                Tbig[k * sm:(k + 1) * sm, h * sm:(h + 1) * sm] += Tsum
        rhs = np.zeros(s * sm)
        for k in range(s):
            rhs[k * sm:k * sm + s] = bet[:, k]
        y = np.linalg.solve(Tbig, rhs).real
        res2 = 0.0
        for k in range(s):
            z = sum(Sbig[k][h] @ y[h * sm:(h + 1) * sm] for h in range(s)).real
            r = z - Vm @ (Vm.T @ z)
            res2 += float(r @ r)
        hist.append(np.sqrt(res2))
        x = np.concatenate([Vm @ y[k * sm:(k + 1) * sm] for k in range(s)])
        if hist[-1] <= eps * nb or sm + s > nbar:
            return x, m, hist
        Vs.append(Q)
    return x, maxit, hist


def modal_bdf(p, s, sample=None):
    """Exact discrete BDF-s solution of a ``workloads.HeatProblem`` whose
    s starting values all equal u0 (scalar recurrence per sine mode; 2D:
    per pair of modes with the eigenvalues of T added, f = 0).  2D with
    sample = (t indices, point indices): only those values."""
    beta, alpha = coefficients(s)
    n, ell, tau, h = p.n, p.ell, p.tau, p.h
    x = np.arange(1, n + 1) * h

    def series(m_k, kap, c0, a, b):
        hist = [c0] * s
        out = np.empty(ell)
        for j in range(1, ell + 1):
            acc = tau * beta * (a * np.cos(b * j * tau) if a != 0.0 else 0.0)
            for q in range(1, s + 1):
                acc += alpha[q - 1] * hist[-q]
            c = acc / (1.0 + tau * beta * kap / m_k)
            hist.append(c)
            out[j - 1] = c
        return out

    if p.dims == 2:
        if p.src_a.size:
            raise ValueError("2D modal oracle supports f = 0 only")
        if sample is not None:                     # values at (t, i) pairs only
            tt, ii = (np.asarray(a) for a in sample)
            yy, xx = ii // n, ii % n
            out = np.zeros(tt.size)
            for (k, m), c0 in p.u0_modes.items():
                kap = _toeplitz_symbol(p.K, k, h) + _toeplitz_symbol(p.K, m, h)
                ser = series(1.0, kap, c0, 0.0, 0.0)
                out += ser[tt] * np.sin(m * np.pi * x[yy]) * np.sin(k * np.pi * x[xx])
            return out
        U = np.zeros((ell, n, n))
        for (k, m), c0 in p.u0_modes.items():
            kap = _toeplitz_symbol(p.K, k, h) + _toeplitz_symbol(p.K, m, h)
            U += series(1.0, kap, c0, 0.0, 0.0)[:, None, None] * \
                np.outer(np.sin(m * np.pi * x), np.sin(k * np.pi * x))[None]
        return U.reshape(ell, n * n)
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
        U += np.outer(series(m_k, kap, c0, a, b), np.sin(k * np.pi * x))
    return U
