"""Pins of the BDF-s oracle (Section 5) against what the mathematics fixes:
the order conditions of the coefficient table, the circulant-plus-rank-s
split of Sigma_s, dense LU of the all-at-once matrix, the scalar recurrence
per sine mode, the convergence order on an ODE with a known solution,
backward Euler at s = 1, and, for the block Galerkin method of the
Proposition, its residual formula against the true residual, exactness on
the full space and Algorithm 2 at s = 1."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import allatonce, bdf, paradiag
from oracle.spatial import problem_matrices, spatial_matrices
from paper_2304_12597_amd import workloads as wl


def _problem(kind, n, ell, s, seed, T=1.0, nu=1.0):
    rng = np.random.default_rng(seed)
    if kind == "fd1":
        M, K = None, wl.fd_laplacian(n, nu)
    else:
        M, K = wl.fem_mass(n), wl.fem_stiffness(n, nu)
    U0 = [rng.standard_normal(n) for _ in range(s)]
    F = rng.standard_normal((ell, n))
    Msp, Ksp = spatial_matrices(M, K, 1)
    return Msp, Ksp, T / ell, U0, F


@pytest.mark.parametrize("s", range(1, 7))
def test_table_order_conditions(s):
    """u_n - sum_j alpha_j u_{n-j} = tau beta u'(t_n) is exact for every
    polynomial of degree <= s and not for degree s + 1 (order exactly s):
    with t_n = 0 and tau = 1, sum_j alpha_j (-j)^q = 0^q - beta q 0^(q-1)."""
    beta, alpha = bdf.BDF[s]
    assert len(alpha) == s

    def defect(q):
        lhs = (Fr(1) if q == 0 else Fr(0)) - sum(a * Fr(-j) ** q for j, a in
                                                 enumerate(alpha, start=1))
        rhs = beta if q == 1 else Fr(0)
        return lhs - rhs
    for q in range(s + 1):
        assert defect(q) == 0, (s, q)
    assert defect(s + 1) != 0


@pytest.mark.parametrize("ell", [8, 12, 16])
@pytest.mark.parametrize("s", range(1, 7))
def test_sigma_split(ell, s):
    """Sigma_s = C_s - [e_1..e_s] A_s [e_{ell-s+1}..e_ell]^T exactly, A_s
    upper triangular with alpha_s on the diagonal and alpha_1 top right."""
    S = bdf.sigma_s(ell, s)
    C = bdf.circulant_cs(ell, s)
    A = bdf.alpha_block(s)
    E = np.eye(ell)[:, :s]
    Et = np.eye(ell)[:, ell - s:]
    assert np.array_equal(S, C - E @ A @ Et.T)
    _, alpha = bdf.coefficients(s)
    assert np.array_equal(np.diag(A), np.full(s, alpha[-1]))
    assert A[0, -1] == alpha[0]
    assert np.array_equal(A, np.triu(A))
    # C_s is circulant: every column is the first one shifted down
    for k in range(ell):
        assert np.array_equal(C[:, k], np.roll(C[:, 0], k))


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("s", range(1, 7))
def test_stepping_matches_dense_lu(kind, s):
    Msp, Ksp, tau, U0, F = _problem(kind, 9, 12, s, 10 * s)
    D = bdf.solve_dense_bdf(Msp, Ksp, tau, s, U0, F)
    S = bdf.step_bdf(Msp, Ksp, tau, s, U0, F)
    assert allatonce.rel_err(S, D) < 1e-12
    R = bdf.apply_bdf(Msp, Ksp, tau, s, D) - bdf.rhs_bdf(Msp, tau, s, U0, F)
    assert np.linalg.norm(R) < 1e-11 * np.linalg.norm(bdf.rhs_bdf(Msp, tau, s, U0, F))


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("s", [2, 4, 6])
def test_modal_recurrence_matches_stepping(kind, s):
    """With u_{1-s} = ... = u_0 = u0 and sine-series data, each sine mode
    follows its own scalar BDF recurrence."""
    p = wl.heat_1d(kind, 31, 24, 1.0, 0.5, np.random.default_rng(s), True)
    Msp, Ksp = problem_matrices(p)
    S = bdf.step_bdf(Msp, Ksp, p.tau, s, [p.u0] * s, p.F)
    assert allatonce.rel_err(bdf.modal_bdf(p, s), S) < 1e-12


@pytest.mark.parametrize("s", range(1, 7))
def test_convergence_order(s):
    """u' = -u + cos t (u = (cos t + sin t)/2 + c e^{-t}) with exact starting
    values: halving tau divides the error at t = 1 by about 2^s."""
    c = 0.7

    def exact(t):
        return 0.5 * (np.cos(t) + np.sin(t)) + c * np.exp(-t)
    Msp, Ksp = spatial_matrices(None, (np.zeros(1), np.ones(1), np.zeros(1)), 1)
    errs = []
    for ell in (16, 32):
        tau = 1.0 / ell
        U0 = [np.array([exact(j * tau)]) for j in range(1 - s, 1)]
        F = np.cos(tau * np.arange(1, ell + 1))[:, None]
        U = bdf.step_bdf(Msp, Ksp, tau, s, U0, F)
        errs.append(abs(U[-1, 0] - exact(1.0)))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - s) < 0.35, (s, errs, rate)


def test_s1_is_backward_euler():
    Msp, Ksp, tau, U0, F = _problem("fem1", 9, 8, 1, 3)
    assert np.allclose(bdf.rhs_bdf(Msp, tau, 1, U0, F), allatonce.rhs(Msp, tau, U0[0], F),
                       rtol=0, atol=1e-15)
    assert allatonce.rel_err(bdf.step_bdf(Msp, Ksp, tau, 1, U0, F),
                             allatonce.step_sparse(Msp, Ksp, tau, U0[0], F)) < 1e-14
    assert np.allclose(bdf.sigma_s(8, 1), allatonce.sigma1(8))


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("s", range(1, 7))
def test_paradiag_bdf_matches_dense_lu(kind, s):
    """The rank-s Sherman-Morrison-Woodbury solve with the s x s block
    capacitance matrix reproduces the all-at-once solution; at s = 1 it is
    Algorithm 1."""
    Msp, Ksp, tau, U0, F = _problem(kind, 7, 16, s, 7 + s)
    D = bdf.solve_dense_bdf(Msp, Ksp, tau, s, U0, F)
    out = bdf.paradiag_bdf(Msp, Ksp, tau, s, U0, F)
    assert allatonce.rel_err(out["U"], D) < 1e-12
    assert allatonce.rel_err(out["U1"], D) > 1e-6        # the correction matters
    if s == 1:
        ref = allatonce.solve_dense(Msp, Ksp, tau, U0[0], F)
        assert allatonce.rel_err(out["U"], ref) < 1e-12
        U1 = paradiag.periodic_solution(Msp, Ksp, tau, U0[0], F)
        assert allatonce.rel_err(out["U1"], U1) < 1e-12


@pytest.mark.parametrize("s", [2, 3, 6])
def test_gamma_reading(s):
    """gamma^(k) must be N e_k with N = F^{-T}[e_{ell-s+1}..e_ell] A_s^T; the
    untransposed A_s e_k (as printed beside theta) does not give the
    solution for s > 1."""
    Msp, Ksp, tau, U0, F = _problem("fd1", 7, 16, s, 3 * s)
    D = bdf.solve_dense_bdf(Msp, Ksp, tau, s, U0, F)
    out = bdf.paradiag_bdf(Msp, Ksp, tau, s, U0, F, gamma_transposed=False)
    assert allatonce.rel_err(out["U"], D) > 1e-4


def test_pins_catch_planted_mistakes(monkeypatch):
    """Plant plausible mistakes in the oracle (CPU only): a sign in the
    table, reversed starting values, a dropped initial-value term."""
    good = dict(bdf.BDF)
    bad = dict(good)
    beta, alpha = good[3]
    bad[3] = (beta, [alpha[0], -alpha[1], alpha[2]])
    monkeypatch.setattr(bdf, "BDF", bad)
    with pytest.raises(AssertionError):
        test_table_order_conditions(3)
    with pytest.raises(AssertionError):
        test_convergence_order(3)
    monkeypatch.setattr(bdf, "BDF", good)

    good_rhs = bdf.rhs_bdf

    def reversed_u0(Msp, tau, s, U0, F):
        return good_rhs(Msp, tau, s, U0[::-1], F)
    monkeypatch.setattr(bdf, "rhs_bdf", reversed_u0)
    Msp, Ksp, tau, U0, F = _problem("fd1", 7, 12, 3, 5)
    Dbad = bdf.solve_dense_bdf(Msp, Ksp, tau, 3, U0, F)
    monkeypatch.setattr(bdf, "rhs_bdf", good_rhs)
    assert allatonce.rel_err(bdf.step_bdf(Msp, Ksp, tau, 3, U0, F), Dbad) > 1e-6

    def no_history(Msp, tau, s, U0, F):     # only alpha_1 u_0 enters row 0
        beta, alpha = bdf.coefficients(s)
        H = tau * beta * np.array(F)
        H[0] += alpha[0] * U0[-1]
        return np.asarray((Msp @ H.T).T)
    monkeypatch.setattr(bdf, "rhs_bdf", no_history)
    Dbad = bdf.solve_dense_bdf(Msp, Ksp, tau, 3, U0, F)
    monkeypatch.setattr(bdf, "rhs_bdf", good_rhs)
    assert allatonce.rel_err(bdf.step_bdf(Msp, Ksp, tau, 3, U0, F), Dbad) > 1e-6


# --------------------------------------------- block Galerkin (Proposition) --

def _block_case(kind, n, s, seed, ell=16):
    Msp, Ksp, tau, U0, F = _problem(kind, n, ell, s, seed)
    P = bdf._pieces(Msp, Ksp, tau, s, U0, F)
    J = bdf.paradiag_bdf(Msp, Ksp, tau, s, U0, F)["J"]
    return Msp, Ksp, tau, U0, F, P, J


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("s", [2, 3])
def test_block_galerkin_residual_formula(kind, s):
    """||(I - I_s (x) V_m V_m^T) S_m y|| of the Proposition is the true
    residual ||J^(s) x_m - b^(s)|| at every m."""
    Msp, Ksp, tau, U0, F, P, J = _block_case(kind, 12, s, 40 + s)
    b = P["b"]
    for m in range(1, 12 // s):
        x, mm, hist = bdf.block_galerkin(Msp, Ksp, tau, s, P, eps=0.0, maxit=m)
        assert mm == m
        true = np.linalg.norm(J @ x - b)
        assert abs(hist[-1] - true) <= 1e-8 * true + 1e-15 * np.linalg.norm(b), (m, hist[-1], true)


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
@pytest.mark.parametrize("s", [2, 3, 4, 6])
def test_block_galerkin_full_space_is_exact(kind, s):
    """Once the block Krylov space is all of R^nbar (m s = nbar) the Galerkin
    solution is the solution, and U solves the all-at-once system."""
    Msp, Ksp, tau, U0, F, P, J = _block_case(kind, 12, s, 50 + s)
    out = bdf.paradiag_bdf(Msp, Ksp, tau, s, U0, F, capacitance="galerkin", eps=1e-14)
    assert out["steps"] <= 12 // s
    D = bdf.solve_dense_bdf(Msp, Ksp, tau, s, U0, F)
    assert allatonce.rel_err(out["U"], D) < 1e-12


def test_block_galerkin_s1_is_algorithm2():
    """At s = 1 the block method is Algorithm 2: the same iterate x_m at
    every m as the Galerkin projection onto K_m(tau M^{-1} K, b) imposed
    directly (alpha = 1, where gamma^(1) is the backward-Euler gamma)."""
    Msp, Ksp, tau, U0, F, P, J = _block_case("fem1", 12, 1, 3)
    cap = paradiag.Capacitance(Msp, Ksp, tau, F.shape[0])
    for m in range(1, 6):
        xb, _, _ = bdf.block_galerkin(Msp, Ksp, tau, 1, P, eps=0.0, maxit=m)
        xf, mf, _ = paradiag.galerkin_projection(cap, Msp, Ksp, tau, P["b"], eps=0.0, maxit=m)
        assert mf == m
        assert np.linalg.norm(xb - xf) <= 1e-10 * np.linalg.norm(xf)


@pytest.mark.parametrize("s", [2, 5])
def test_modal_recurrence_2d_matches_stepping(s):
    """2D (K = I (x) T + T (x) I, f = 0): each pair of sine modes follows the
    scalar BDF recurrence with the sum of the two eigenvalues of T."""
    p = wl.heat_2d(15, 16, 0.1, 1.0, np.random.default_rng(s))
    Msp, Ksp = problem_matrices(p)
    S = bdf.step_bdf(Msp, Ksp, p.tau, s, [p.u0] * s, p.F)
    assert allatonce.rel_err(bdf.modal_bdf(p, s), S) < 1e-12


@pytest.mark.parametrize("s", [1, 2, 3])
def test_modal_bdf_sampled_branch_matches_full(s):
    """The point-by-point (sampled) branch of the 2D per-mode BDF recurrence,
    which grades full-size GPU results, equals the full-array branch at the
    same (t, point) pairs, including the first and last time rows and grid
    corners; the full branch is itself pinned to sequential stepping."""
    p = wl.heat_2d(15, 16, 0.1, 1.0, np.random.default_rng(40 + s))
    full = bdf.modal_bdf(p, s)
    rng = np.random.default_rng(s)
    tt = rng.integers(0, p.ell, 500)
    ii = rng.integers(0, p.nbar, 500)
    tt[:4] = [0, 0, p.ell - 1, p.ell - 1]
    ii[:4] = [0, p.nbar - 1, p.n - 1, p.nbar - p.n]
    samp = bdf.modal_bdf(p, s, (tt, ii))
    assert np.allclose(samp, full[tt, ii], rtol=1e-13, atol=1e-15 * np.abs(full).max())
    # a transposed point index (x and y swapped) would not match
    swapped = (ii % p.n) * p.n + ii // p.n
    assert not np.allclose(full[tt, swapped], full[tt, ii])
