"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute-force
sums, dense eigen-decompositions, dense LU of the all-at-once matrix, closed
forms, the values printed in the paper (tests/golden), or invariants.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401  (sp.linalg)

from oracle import allatonce, dst, modal, paradiag
from oracle.spatial import problem_matrices, spatial_matrices
from paper_2304_12597_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_problem(kind, n, ell, seed, T=1.0, nu=1.0):
    rng = np.random.default_rng(seed)
    if kind == "fd1":
        M, K = None, wl.fd_laplacian(n, nu)
    else:
        M, K = wl.fem_mass(n), wl.fem_stiffness(n, nu)
    u0 = rng.standard_normal(n)
    F = rng.standard_normal((ell, n))
    Msp, Ksp = spatial_matrices(M, K, 1)
    return M, K, Msp, Ksp, T / ell, u0, F


# ---------------------------------------------------------------- Fourier --

def test_fft_matches_brute_force_dft():
    """numpy's FFT along time equals the DFT sum with omega = e^{-2 pi i/ell}
    (the un-normalised transform of Section 2)."""
    rng = np.random.default_rng(0)
    ell, nb = 8, 3
    X = rng.standard_normal((ell, nb)) + 1j * rng.standard_normal((ell, nb))
    ref = np.zeros_like(X)
    for k in range(ell):
        for t in range(ell):
            ref[k] += X[t] * np.exp(-2j * np.pi * t * k / ell)
    assert np.allclose(np.fft.fft(X, axis=0), ref, atol=1e-13)
    assert np.allclose(paradiag.dft_matrix(ell) @ X, ref, atol=1e-13)
    # inverse: F^{-1} = conj(F) / ell
    Fm = paradiag.dft_matrix(ell)
    assert np.allclose(np.linalg.inv(Fm), Fm.conj() / ell, atol=1e-14)


@pytest.mark.parametrize("ell", [1, 2, 5, 8, 16])
@pytest.mark.parametrize("alpha", [1.0, 1e-2])
def test_circulant_eigenvalues(ell, alpha):
    """pi = alpha^(1/ell) F C_1 e_1 diagonalises C_alpha with the scaled DFT
    (Sections 2 and 4), and gamma = F^{-T} e_ell."""
    Fm = paradiag.dft_matrix(ell)
    pi, gamma = paradiag.circulant_eigs(ell, alpha)
    C = paradiag.circulant_c1(ell, alpha)
    w = alpha ** (1.0 / ell)
    D = np.diag(w ** np.arange(ell))
    # C_alpha = D^{-1} F^{-1} Pi F D
    recon = np.linalg.inv(D) @ np.linalg.inv(Fm) @ np.diag(pi) @ Fm @ D
    assert np.allclose(recon, C, atol=1e-12)
    # eigenvalues match a dense eigen-solver (as multisets)
    ev = np.linalg.eigvals(C)
    for p in pi:
        assert np.min(np.abs(ev - p)) < 1e-9
    # F C_1 e_1 literally (alpha = 1 form of Algorithm 1)
    C1 = paradiag.circulant_c1(ell, 1.0)
    assert np.allclose(w * (Fm @ C1[:, 0]), pi, atol=1e-12)
    el = np.zeros(ell); el[-1] = 1.0
    assert np.allclose(np.linalg.solve(Fm.T, el), gamma, atol=1e-13)
    if alpha == 1.0:
        assert np.allclose(gamma, pi / ell)   # Appendix


def test_sigma1_split():
    """Sigma_1 = C_1 - e_1 e_ell^T = C_alpha - alpha e_1 e_ell^T."""
    ell = 6
    e1 = np.zeros(ell); e1[0] = 1
    el = np.zeros(ell); el[-1] = 1
    for a in (1.0, 0.3):
        assert np.array_equal(allatonce.sigma1(ell),
                              paradiag.circulant_c1(ell, a) - a * np.outer(e1, el))


# ------------------------------------------------------ all-at-once (O1/O2) --

@pytest.mark.parametrize("kind", ["fd1", "fem1"])
def test_stepping_matches_dense_lu(kind):
    """O1 (C Thomas stepping) equals O2 (dense LU of the Kronecker matrix)."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem(kind, 7, 8, 1)
    U2 = allatonce.solve_dense(Msp, Ksp, tau, u0, F)
    U1 = allatonce.step_1d(M, K, tau, u0, F)
    assert allatonce.rel_err(U1, U2) < 1e-13
    _, rr = allatonce.residual(Msp, Ksp, tau, u0, F, U2)
    assert rr < 1e-13
    U1s = allatonce.step_sparse(Msp, Ksp, tau, u0, F)
    assert allatonce.rel_err(U1s, U2) < 1e-13


def test_stepping_2d_matches_dense_lu():
    n, ell = 3, 4
    K = wl.fd_laplacian(n, 0.7)
    Msp, Ksp = spatial_matrices(None, K, 2)
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal(n * n)
    F = rng.standard_normal((ell, n * n))
    U2 = allatonce.solve_dense(Msp, Ksp, 0.1, u0, F)
    U1 = allatonce.step_sparse(Msp, Ksp, 0.1, u0, F)
    assert allatonce.rel_err(U1, U2) < 1e-13
    # K = I (x) T + T (x) I
    Td = wl.dense_tridiag(K)
    assert np.allclose(Ksp.toarray(), np.kron(np.eye(n), Td) + np.kron(Td, np.eye(n)))


def test_dense_matrix_is_block_bidiagonal():
    """The Kronecker matrix has (M + tau K) on the diagonal and -M on the
    first block subdiagonal (the backward-Euler step)."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem("fem1", 4, 3, 2)
    A = allatonce.dense_matrix(Msp, Ksp, tau, 3)
    Md = wl.dense_tridiag(M)
    Ad = Md + tau * wl.dense_tridiag(K)
    assert np.allclose(A[:4, :4], Ad) and np.allclose(A[4:8, :4], -Md)
    assert np.allclose(A[:4, 4:8], 0) and np.allclose(A[8:, 4:8], -Md)


# ---------------------------------------------------------------- modal (O3) --

@pytest.mark.parametrize("kind", ["fd1", "fem1"])
def test_modal_matches_dense_lu(kind):
    rng = np.random.default_rng(11)
    p = wl.heat_1d(kind, 15, 8, 1.0, 0.5, rng, True)
    Msp, Ksp = problem_matrices(p)
    U2 = allatonce.solve_dense(Msp, Ksp, p.tau, p.u0, p.F)
    U3 = modal.modal_solution(p)
    assert allatonce.rel_err(U3, U2) < 1e-12
    ii = np.array([0, 3, 14, 7]); tt = np.array([0, 7, 3, 5])
    assert np.allclose(modal.modal_sample(p, tt, ii), U3[tt, ii], atol=1e-13)


def test_modal_2d_matches_stepping():
    p = wl.heat_2d(15, 8, 0.1, 1.0, np.random.default_rng(3))
    U3 = modal.modal_solution(p)
    U1 = allatonce.step(p)
    assert allatonce.rel_err(U3, U1) < 1e-12
    ii = np.array([0, 17, 224]); tt = np.array([0, 7, 2])
    assert np.allclose(modal.modal_sample(p, tt, ii), U3[tt, ii], atol=1e-13)


def test_sine_mode_decay_closed_form():
    """f = 0, u0 = s_k: u_j = (1 + tau mu_k)^(-j) s_k with
    mu_k = (4 nu/h^2) sin^2(k pi h / 2) for finite differences; mu_k is
    checked against a dense eigen-solver."""
    n, ell, nu, k = 31, 16, 0.8, 5
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    s = np.sin(k * np.pi * x)
    mu = 4 * nu / h**2 * np.sin(k * np.pi * h / 2) ** 2
    K = wl.fd_laplacian(n, nu)
    ev = np.linalg.eigvalsh(wl.dense_tridiag(K))
    assert np.min(np.abs(ev - mu)) < 1e-9 * mu
    p = wl.HeatProblem("fd1", n, ell, 1.0, nu, None, K, s, np.zeros((ell, n)),
                       {k: 1.0})
    U = modal.modal_solution(p)
    tau = 1.0 / ell
    ref = np.outer((1 + tau * mu) ** -np.arange(1, ell + 1), s)
    assert np.allclose(U, ref, rtol=1e-13, atol=1e-15)
    U1 = allatonce.step(p)
    assert allatonce.rel_err(U1, ref) < 1e-12


# ------------------------------------------------- ParaDiag (Alg. 1 / 3, O4) --

def _reassemble(Msp, Ksp, tau, u0, F, alpha, cap_method="dense"):
    """The Sherman-Morrison-Woodbury assembly of Section 2 (eq. SMW_U; Section
    4 for alpha < 1) from the oracle's separately defined pieces:
    U = U_1 - w W F^{-T} D_alpha^{-1} with W_i = P_i^{-1} M x, x = J^{-1} b."""
    ell = F.shape[0]
    cap = paradiag.Capacitance(Msp, Ksp, tau, ell, alpha)
    U1 = paradiag.periodic_solution(Msp, Ksp, tau, u0, F, alpha)
    b = paradiag.capacitance_rhs(U1, alpha)
    x = paradiag.capacitance_solution(cap, b, cap_method)
    Mx = Msp @ x
    W = paradiag.shifted_solutions(cap, np.tile(Mx.astype(np.complex128), (ell, 1)))
    w = alpha ** (1.0 / ell)
    scale = w ** np.arange(ell)
    U = U1 - w * np.fft.ifft(W, axis=0) / scale[:, None]
    return dict(cap=cap, U1=U1, b=b, x=x, W=W, U=U)


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("alpha", [1.0, 1e-2])
@pytest.mark.parametrize("cap", ["dense", "gmres"])
def test_smw_pieces_reassemble_dense_lu(kind, alpha, cap):
    """The pieces, each from its own definition, satisfy the identities that
    connect them in Algorithm 1 / 3: the blockwise solves of the spectrum of
    G are U_1 in Fourier variables (U_1 by stepping, no transform), b is
    both a time slice of U_1 and L F^{-T} e_ell, x = alpha^((ell-1)/ell) u_ell,
    and U_1 - w W F^{-T} D_alpha^{-1} is the dense-LU solution."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem(kind, 7, 8, 3)
    ell = F.shape[0]
    U2 = allatonce.solve_dense(Msp, Ksp, tau, u0, F)
    out = _reassemble(Msp, Ksp, tau, u0, F, alpha, cap)
    pieces = out["cap"]
    L = paradiag.shifted_solutions(pieces, paradiag.rhs_spectrum(Msp, tau, u0, F, alpha))
    w = alpha ** (1.0 / ell)
    kappa = alpha ** (-(ell - 1) / ell)
    assert allatonce.rel_err(np.fft.ifft(L, axis=0).real / (w ** np.arange(ell))[:, None],
                             out["U1"]) < 1e-13 * kappa
    assert np.allclose((pieces.gamma[:, None] * L).sum(axis=0), out["b"], rtol=1e-11,
                       atol=1e-13)
    assert np.max(np.abs(out["U"].imag)) < 1e-12
    assert allatonce.rel_err(out["U"].real, U2) < 1e-11
    assert np.allclose(out["x"], alpha ** ((ell - 1) / ell) * U2[-1],
                       rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("alpha", [1.0, 1e-2])
def test_smw_dense_matches_dense_lu(kind, alpha):
    M, K, Msp, Ksp, tau, u0, F = _random_problem(kind, 5, 6, 4)
    U2 = allatonce.solve_dense(Msp, Ksp, tau, u0, F)
    U4 = paradiag.smw_dense(Msp, Ksp, tau, u0, F, alpha=alpha)
    assert np.max(np.abs(U4.imag)) < 1e-11
    assert allatonce.rel_err(U4.real, U2) < 1e-11


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("alpha", [1e-2, 1e-6, 1.0])
def test_alpha_first_term_solves_alpha_circulant_system(kind, alpha):
    """Algorithm 3: U_1 is the exact solution of the all-at-once system with
    Sigma_1 replaced by C_alpha (dense LU of I (x) (M + tau K) - C_alpha (x) M),
    and its residual in the original system is -alpha M u_ell in the first
    time row and zero elsewhere (C_alpha - Sigma_1 = alpha e_1 e_ell^T)."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem(kind, 7, 8, 21)
    ell, nbar = F.shape
    U1 = paradiag.periodic_solution(Msp, Ksp, tau, u0, F, alpha)
    Md = Msp.toarray()
    A = np.kron(np.eye(ell), Md + tau * Ksp.toarray()) - np.kron(
        paradiag.circulant_c1(ell, alpha), Md)
    G = allatonce.rhs(Msp, tau, u0, F)
    U1_lu = np.linalg.solve(A, G.reshape(-1)).reshape(ell, nbar)
    assert allatonce.rel_err(U1, U1_lu) < 1e-13
    R, _ = allatonce.residual(Msp, Ksp, tau, u0, F, U1_lu)
    expect = np.zeros_like(R)
    expect[0] = -alpha * (Msp @ U1_lu[-1])
    assert np.allclose(R, expect, rtol=0, atol=1e-12 * np.linalg.norm(G))


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
def test_alpha_early_exit_decision(kind):
    """Algorithm 3's test: with eps just above the first term's residual
    ratio ||G - A(U_1)||_F / ||M U_1||_F, U_1 is accepted; just below it, it
    is not.  The ratio has the closed form alpha ||M u_ell|| / ||M U_1||."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem(kind, 7, 8, 22)
    alpha = 1e-6
    U1 = paradiag.periodic_solution(Msp, Ksp, tau, u0, F, alpha)
    _, rel = allatonce.residual(Msp, Ksp, tau, u0, F, U1)
    G = allatonce.rhs(Msp, tau, u0, F)
    MU1 = np.asarray((Msp @ U1.T).T)
    ratio = rel * np.linalg.norm(G) / np.linalg.norm(MU1)
    assert np.isclose(ratio, alpha * np.linalg.norm(Msp @ U1[-1]) / np.linalg.norm(MU1),
                      rtol=1e-6)
    assert paradiag.first_term_accepted(Msp, Ksp, tau, u0, F, U1, 1.01 * ratio)
    assert not paradiag.first_term_accepted(Msp, Ksp, tau, u0, F, U1, 0.99 * ratio)


def test_smw_pieces_2d_match_stepping():
    p = wl.heat_2d(7, 8, 0.1, 1.0, np.random.default_rng(9))
    Msp, Ksp = problem_matrices(p)
    out = _reassemble(Msp, Ksp, p.tau, p.u0, p.F, 1.0, "gmres")
    assert allatonce.rel_err(out["U"].real, allatonce.step(p)) < 1e-11


def test_b_is_last_column_of_periodic_solution():
    """b = L F^{-T} e_ell (the gamma-weighted sum of the blockwise solves of
    the spectrum) is the last column of the solution of the circulant
    (periodic) system (M + tau K) U - M U C_1^T = G, computed here by dense
    LU, and the oracle's stepping form of U_1 agrees with it."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem("fem1", 6, 8, 6)
    ell, n = F.shape
    G = allatonce.rhs(Msp, tau, u0, F)
    Md = Msp.toarray()
    Ad = Md + tau * Ksp.toarray()
    C1 = paradiag.circulant_c1(ell)
    Acirc = np.kron(np.eye(ell), Ad) - np.kron(C1, Md)
    Uper = np.linalg.solve(Acirc, G.reshape(-1)).reshape(ell, n)
    cap = paradiag.Capacitance(Msp, Ksp, tau, ell)
    L = paradiag.shifted_solutions(cap, paradiag.rhs_spectrum(Msp, tau, u0, F))
    b = (cap.gamma[:, None] * L).sum(axis=0)
    assert np.allclose(b, Uper[-1], rtol=1e-11, atol=1e-13)
    U1 = paradiag.periodic_solution(Msp, Ksp, tau, u0, F)
    assert np.allclose(U1, Uper, rtol=1e-11, atol=1e-13)
    assert np.allclose(paradiag.capacitance_rhs(U1), Uper[-1], rtol=1e-11, atol=1e-13)


def test_capacitance_on_sine_vectors():
    """On a sine vector with generalised eigenvalue mu (K s = mu M s),
    J_ell s = a^ell / (a^ell - alpha) s with a = 1 + tau mu."""
    n, ell = 15, 8
    for kind in ("fd1", "fem1"):
        M, K, Msp, Ksp, tau, _, _ = _random_problem(kind, n, ell, 7)
        h = 1.0 / (n + 1)
        k = 3
        s = np.sin(k * np.pi * np.arange(1, n + 1) * h)
        Ms = Msp @ s
        mu = (Ksp @ s)[4] / Ms[4]
        assert np.allclose(Ksp @ s, mu * Ms)
        for alpha in (1.0, 0.1):
            cap = paradiag.Capacitance(Msp, Ksp, tau, ell, alpha)
            a = 1 + tau * mu
            Js = cap.matvec(s)
            assert np.allclose(Js, a**ell / (a**ell - alpha) * s, rtol=1e-12)


def test_theorem1_hermitian_pd_and_bound():
    """Theorem 1 (K SPD, M = I): J_ell Hermitian positive definite and
    kappa(J_ell) <= 1 + 1/(tau lambda_min(K))."""
    for ell in (1, 2, 7, 8):
        n = 9
        K = wl.fd_laplacian(n, 0.05)
        Msp, Ksp = spatial_matrices(None, K, 1)
        tau = 1.0 / ell
        J = paradiag.Capacitance(Msp, Ksp, tau, ell).dense()
        assert np.allclose(J, J.conj().T, atol=1e-12)
        ev = np.linalg.eigvalsh(J)
        assert ev.min() > 0
        lam_min = np.linalg.eigvalsh(Ksp.toarray()).min()
        assert ev.max() / ev.min() <= paradiag.theorem1_bound(tau, lam_min) + 1e-12


def _read_table(path):
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_table1_bounds():
    """Table 1 of Section 6.1 from lambda_min(K) = (8/h^2) sin^2(pi/(2(n+1)))."""
    rows = _read_table(os.path.join(GOLDEN, "table1.txt"))
    assert len(rows) == 9
    for nbar, ell, printed in rows:
        n = int(round(np.sqrt(int(nbar))))
        assert n * n == int(nbar)
        bound = paradiag.theorem1_bound(1.0 / int(ell),
                                        paradiag.lambda_min_2d_laplacian(n))
        assert abs(bound - float(printed)) < 1e-3, (nbar, ell, bound, printed)


def test_lambda_min_closed_form_matches_eigensolver():
    n = 12
    K = wl.fd_laplacian(n, 1.0)
    _, Ksp = spatial_matrices(None, K, 2)
    ev = np.linalg.eigvalsh(Ksp.toarray())
    assert abs(ev.min() - paradiag.lambda_min_2d_laplacian(n)) < 1e-9 * ev.min()


def test_j_spectrum_section61():
    """[lambda_min(J), lambda_max(J)] in [1, 1.004] for all Table 1 sizes;
    the extreme-eigenvalue sums are first checked against a dense
    eigen-decomposition of J on a small 2D problem."""
    lo_g, hi_g = [float(r[1]) for r in _read_table(os.path.join(GOLDEN, "j_spectrum.txt"))]
    n, ell = 5, 8
    K = wl.fd_laplacian(n, 1.0)
    Msp, Ksp = spatial_matrices(None, K, 2)
    tau = 1.0 / ell
    J = paradiag.Capacitance(Msp, Ksp, tau, ell).dense()
    ev = np.linalg.eigvalsh(0.5 * (J + J.conj().T))
    kev = np.linalg.eigvalsh(Ksp.toarray())
    lo, hi = paradiag.j_extreme_eigs(tau, ell, kev.min(), kev.max())
    assert abs(lo.real - ev.min()) < 1e-12 and abs(hi.real - ev.max()) < 1e-12
    for nbar, ell_s, _ in _read_table(os.path.join(GOLDEN, "table1.txt")):
        n = int(round(np.sqrt(int(nbar))))
        ell = int(ell_s)
        h = 1.0 / (n + 1)
        lmin = paradiag.lambda_min_2d_laplacian(n)
        lmax = 8.0 / h**2 * np.cos(np.pi / (2 * (n + 1)))**2
        lo, hi = paradiag.j_extreme_eigs(1.0 / ell, ell, lmin, lmax)
        assert abs(lo.imag) < 1e-12 and abs(hi.imag) < 1e-12
        assert lo_g <= lo.real <= hi.real <= hi_g


def test_gmres_oracle_matches_dense():
    rng = np.random.default_rng(0)
    A = np.eye(20) + 0.1 * rng.standard_normal((20, 20))
    b = rng.standard_normal(20)
    x, its, hist = paradiag.gmres(lambda v: A @ v, b, tol=1e-14, maxit=40)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10)
    assert hist[-1] <= 1e-13 * np.linalg.norm(b) * 10


def _section61_problem(n, ell):
    p = wl.heat_2d(n, ell, 1.0, 1.0, np.random.default_rng(1))
    x = np.arange(1, n + 1) / (n + 1)
    X, Y = np.meshgrid(x, x)
    p.u0 = (X * Y * (X - 1) * (1 - Y)).reshape(-1)
    return p


def test_one_inner_iteration_suffices_2d():
    """Section 6.1: for the 2D heat example J_ell is a tiny perturbation of
    I, so the Krylov solve reaches 1e-8 almost at once (checked here with
    GMRES on a scaled-down grid: at most 2 iterations)."""
    n, ell = 15, 32
    p = _section61_problem(n, ell)
    Msp, Ksp = problem_matrices(p)
    cap = paradiag.Capacitance(Msp, Ksp, p.tau, ell)
    b = paradiag.capacitance_rhs(paradiag.periodic_solution(Msp, Ksp, p.tau, p.u0, p.F))
    _, its, _ = paradiag.gmres(lambda v: cap.matvec(v).real, b, tol=1e-8)
    assert its <= 2


def _paper_projection(cap, Msp, Ksp, tau, b, m):
    """Algorithm 2's small system and residual as the paper writes them
    (eq. compute_ym and eq. compute_resnorm): S_i = (lambda_i I + T_m)^{-1},
    h_i = P_i^{-1} M v_{m+1}, with the Arnoldi data of K_m(tau M^{-1} K, b).
    Returns (y, residual, and the two printed variants of the residual that
    drop gamma_i or the tau in t_{m+1,m})."""
    Mlu = sp.linalg.splu(Msp.tocsc())
    V = [b / np.linalg.norm(b)]
    Tm = np.zeros((m + 1, m))
    for j in range(m):
        w = tau * Mlu.solve(Ksp @ V[j])
        for k in range(j + 1):
            Tm[k, j] = V[k] @ w
            w = w - Tm[k, j] * V[k]
        for k in range(j + 1):           # second pass (as the oracle's basis)
            c = V[k] @ w
            Tm[k, j] += c
            w = w - c * V[k]
        Tm[j + 1, j] = np.linalg.norm(w)
        V.append(w / Tm[j + 1, j])
    Vm = np.array(V[:m]).T
    t = Tm[m, m - 1]
    lam = 1.0 - cap.pi
    em = np.eye(m)[-1]
    e1 = np.eye(m)[0] * np.linalg.norm(b)
    Z = np.eye(m, dtype=complex)
    S, H = [], []
    for i, g in enumerate(cap.gamma):
        Si = np.linalg.inv(lam[i] * np.eye(m) + Tm[:m, :m])
        hi = cap.solve_shifted(i, Msp @ V[m])
        Z += cap.weight * g * (np.eye(m) - t * np.outer(Vm.T @ hi, em)) @ Si
        S.append(Si)
        H.append(hi)
    y = np.linalg.solve(Z, e1).real
    with_g = sum(g * H[i] * (S[i][-1] @ y) for i, g in enumerate(cap.gamma))
    res = abs(t) * cap.weight * np.linalg.norm(with_g - Vm @ (Vm.T @ with_g))
    no_gamma = sum(H[i] * (S[i][-1] @ y) for i in range(len(H)))
    r_no_gamma = abs(t) * cap.weight * np.linalg.norm(no_gamma - Vm @ (Vm.T @ no_gamma))
    r_no_tau = abs(t / tau) * cap.weight * np.linalg.norm(with_g - Vm @ (Vm.T @ with_g))
    return y, res, r_no_gamma, r_no_tau


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("alpha", [1.0, 1e-2])
def test_projection_formulas_match_direct_galerkin(kind, alpha):
    """Algorithm 2's small system (eq. compute_ym, from the shifted Arnoldi
    relation) gives the same iterate as the Galerkin condition imposed
    directly with J_ell applied to the basis (the oracle), and its residual
    formula (eq. compute_resnorm, with gamma_i and the alpha weight) equals
    the oracle's directly computed ||J x_m - b|| at every m; the two printed
    variants it replaces (no gamma_i in the residual line, and t_{m+1,m}
    without tau for the Krylov space of K) do not."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem(kind, 9, 8, 31)
    cap = paradiag.Capacitance(Msp, Ksp, tau, F.shape[0], alpha)
    b = paradiag.capacitance_rhs(paradiag.periodic_solution(Msp, Ksp, tau, u0, F, alpha), alpha)
    for m_max in (1, 2, 3, 5):
        x, m, hist = paradiag.galerkin_projection(cap, Msp, Ksp, tau, b, eps=0.0, maxit=m_max)
        assert m == m_max
        direct = np.linalg.norm(cap.matvec(x).real - b)
        assert np.isclose(hist[-1], direct, rtol=1e-12, atol=1e-15 * np.linalg.norm(b))
        y, res, r_no_gamma, r_no_tau = _paper_projection(cap, Msp, Ksp, tau, b, m_max)
        Vm = np.linalg.qr(np.array([np.linalg.matrix_power(
            tau * np.linalg.solve(Msp.toarray(), Ksp.toarray()), j) @ b
            for j in range(m_max)]).T)[0]
        assert np.linalg.norm(x - Vm @ (Vm.T @ x)) < 1e-9 * np.linalg.norm(x)
        assert np.isclose(res, direct, rtol=1e-7, atol=1e-14 * np.linalg.norm(b))
        if m_max == 2:
            assert not np.isclose(r_no_gamma, direct, rtol=1e-2)
            assert not np.isclose(r_no_tau, direct, rtol=1e-2)


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
def test_projection_reaches_the_exact_solution(kind):
    """With the whole space (m = nbar) the projection returns the exact x,
    and x = alpha^((ell-1)/ell) u_ell (the last time step of the all-at-once
    solution)."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem(kind, 7, 8, 32)
    alpha = 1e-2
    ell = F.shape[0]
    cap = paradiag.Capacitance(Msp, Ksp, tau, ell, alpha)
    b = paradiag.capacitance_rhs(paradiag.periodic_solution(Msp, Ksp, tau, u0, F, alpha), alpha)
    x, m, _ = paradiag.galerkin_projection(cap, Msp, Ksp, tau, b, eps=1e-14, maxit=7)
    U2 = allatonce.solve_dense(Msp, Ksp, tau, u0, F)
    assert np.allclose(x, alpha ** ((ell - 1) / ell) * U2[-1], rtol=1e-10, atol=1e-12)


def test_projection_one_iteration_suffices_2d():
    """Section 6.1 states that one iteration of Algorithm 2 is enough for the
    2D heat example; on a scaled-down grid the first residual check is below
    1e-8 ||b||."""
    n, ell = 15, 32
    p = _section61_problem(n, ell)
    Msp, Ksp = problem_matrices(p)
    cap = paradiag.Capacitance(Msp, Ksp, p.tau, ell)
    b = paradiag.capacitance_rhs(paradiag.periodic_solution(Msp, Ksp, p.tau, p.u0, p.F))
    _, m, hist = paradiag.galerkin_projection(cap, Msp, Ksp, p.tau, b, eps=1e-8)
    assert m == 1 and hist[0] <= 1e-8 * np.linalg.norm(b)


# ------------------------------------------------------- planted mistakes --

def test_pins_catch_planted_mistakes(monkeypatch):
    """Plant plausible mistakes in the oracle (CPU only) and check that the
    pins reject each of them: the reassembly against dense LU, and the
    blockwise solves of the spectrum against U_1 by stepping."""
    M, K, Msp, Ksp, tau, u0, F = _random_problem("fem1", 7, 8, 12)
    ell = F.shape[0]
    U2 = allatonce.solve_dense(Msp, Ksp, tau, u0, F)
    good = paradiag.circulant_eigs

    def conj_pi(ell, alpha=1.0):       # wrong sign in the exponent of pi
        p, g = good(ell, alpha)
        return p.conj(), g

    def conj_gamma(ell, alpha=1.0):    # gamma = F^{-1} e_ell instead of F^{-T}..
        p, g = good(ell, alpha)
        return p, g.conj()

    for bad in (conj_pi, conj_gamma):
        monkeypatch.setattr(paradiag, "circulant_eigs", bad)
        out = _reassemble(Msp, Ksp, tau, u0, F, 1.0)
        assert allatonce.rel_err(out["U"].real, U2) > 1e-6
        monkeypatch.setattr(paradiag, "circulant_eigs", good)
    # a conjugated pi also breaks the link between the spectrum's solves and U_1
    monkeypatch.setattr(paradiag, "circulant_eigs", conj_pi)
    cap = paradiag.Capacitance(Msp, Ksp, tau, ell)
    monkeypatch.setattr(paradiag, "circulant_eigs", good)
    L = paradiag.shifted_solutions(cap, paradiag.rhs_spectrum(Msp, tau, u0, F))
    U1 = paradiag.periodic_solution(Msp, Ksp, tau, u0, F)
    assert allatonce.rel_err(np.fft.ifft(L, axis=0).real, U1) > 1e-6
    # dropping the rank-one correction (the circulant preconditioner alone)
    assert allatonce.rel_err(U1, U2) > 1e-6
    # forgetting the mass matrix in the capacitance matrix
    good_mv = paradiag.Capacitance.matvec

    def no_mass(self, v):
        acc = sum(g * self.solve_shifted(i, v) for i, g in enumerate(self.gamma))
        return v + self.weight * acc
    monkeypatch.setattr(paradiag.Capacitance, "matvec", no_mass)
    out = _reassemble(Msp, Ksp, tau, u0, F, 1.0, "gmres")
    assert allatonce.rel_err(out["U"].real, U2) > 1e-6
    monkeypatch.setattr(paradiag.Capacitance, "matvec", good_mv)
    # a wrap-around term without alpha in the stepping form of U_1
    good_ps = paradiag.periodic_solution
    U1a = good_ps(Msp, Ksp, tau, u0, F, 1e-2)
    U1b = good_ps(Msp, Ksp, tau, u0, F, 1.0)
    assert allatonce.rel_err(U1b, U1a) > 1e-6


# ------------------------------------------------------------------ DST-I --

def test_sine_matrix_orthogonal_large():
    """S S = I to float64 rounding at a size where unreduced phases fail."""
    n = 2047
    S = dst.sine_matrix(n)
    assert np.max(np.abs(S @ S - np.eye(n))) < 1e-14
    assert np.array_equal(S, S.T)


def test_sine_matrix_diagonalises_toeplitz():
    n = 13
    S = dst.sine_matrix(n)
    assert np.allclose(S @ S, np.eye(n), atol=1e-13)
    assert np.allclose(S, S.T)
    T = wl.dense_tridiag(wl.fd_laplacian(n, 1.0))
    D = S @ T @ S
    assert np.allclose(D, np.diag(np.diag(D)), atol=1e-9)
    assert np.allclose(np.sort(np.diag(D)), np.linalg.eigvalsh(T))
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, n))
    assert np.allclose(dst.dst1(dst.dst1(x)), x)
