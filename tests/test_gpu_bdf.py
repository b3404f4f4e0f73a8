"""GPU parity of the BDF-s path (bdf_order = s in 2..6, Section 5): whole
solves against the oracle's stepping and exact modal recurrence, the
stages (h transform, block capacitance product, capacitance solve,
residual) against the oracle's pieces, and the block Galerkin method
(krylov = PD_KRYLOV_FOM) against the oracle's."""
import numpy as np
import pytest

from oracle import allatonce, bdf
from oracle.spatial import problem_matrices, spatial_matrices
from paper_2304_12597_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=dev())


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _problem(kind, n, ell, s, seed, T_=1.0, nu=1.0):
    """Random data (not a sine series): s distinct starting values."""
    rng = np.random.default_rng(seed)
    if kind == "fd1":
        M, K = None, wl.fd_laplacian(n, nu)
    else:
        M, K = wl.fem_mass(n), wl.fem_stiffness(n, nu)
    U0 = rng.standard_normal((s, n))
    F = rng.standard_normal((ell, n))
    return M, K, T_ / ell, U0, F


def _plan(lib, n, ell, tau, M, K, s, **kw):
    return lib.paradiag_plan_create(n, ell, tau, M, K, bdf_order=s, stream=_stream(), **kw)


def _solve(lib, n, ell, tau, M, K, s, U0, F, tol=1e-12, **kw):
    plan = _plan(lib, n, ell, tau, M, K, s, check_residual=1, **kw)
    try:
        U = torch.empty((ell, n), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(U0), T(F), U, tol)
        torch.cuda.synchronize()
        return U.cpu().numpy(), info
    finally:
        lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("kind,n,ell,s,tol", [
    ("fd1", 15, 16, 2, 1e-10), ("fem1", 15, 16, 3, 1e-10), ("fd1", 63, 32, 4, 1e-10),
    ("fem1", 63, 64, 5, 1e-10), ("fd1", 127, 16, 6, 1e-10), ("fem1", 255, 128, 2, 1e-10),
    ("fd1", 1000, 64, 3, 1e-10), ("fem1", 2047, 32, 6, 1e-10), ("fd1", 2, 4, 2, 1e-10),
    ("fem1", 3, 8, 4, 1e-10), ("fd1", 5, 16, 6, 1e-10), ("fem1", 8191, 16, 3, 1e-9)])
def test_bdf_solve_matches_stepping(lib, kind, n, ell, s, tol):
    """Ragged and power-of-two n, every order: U against sequential BDF
    stepping (sparse LU), #PinT = iterations + 2, residual reported.  Random
    data excites every mode, so two correct float64 solvers differ by up to
    about kappa u (kappa = tau beta lambda_max(M^{-1} K) ~ 3e7 for the FEM
    n = 8191, ell = 16 case: tol 1e-9 there)."""
    M, K, tau, U0, F = _problem(kind, n, ell, s, 100 * s + n)
    U, info = _solve(lib, n, ell, tau, M, K, s, U0, F)
    Msp, Ksp = spatial_matrices(M, K, 1)
    ref = bdf.step_bdf(Msp, Ksp, tau, s, list(U0), F)
    err = allatonce.rel_err(U, ref)
    assert err < tol, (err, info.as_dict())
    assert info.pint_loops == info.gmres_iters + 2
    assert 0 <= info.rel_residual < 1e-10


@pytest.mark.parametrize("s", [2, 3, 4, 5, 6])
def test_bdf_matches_oracle_smw(lib, s):
    """The same pieces as the oracle's rank-s SMW solve: b^(s) through the
    capacitance solve gives the oracle's x, and U agrees with its U."""
    n, ell = 15, 16
    M, K, tau, U0, F = _problem("fem1", n, ell, s, 7 * s)
    Msp, Ksp = spatial_matrices(M, K, 1)
    ref = bdf.paradiag_bdf(Msp, Ksp, tau, s, list(U0), F)
    plan = _plan(lib, n, ell, tau, M, K, s)
    try:
        x = torch.empty(s * n, dtype=torch.float64, device=dev())
        its, rr = lib.paradiag_capacitance_solve(plan, T(ref["b"]), x, 1e-13)
        Jv = torch.empty(s * n, dtype=torch.float64, device=dev())
        v = np.random.default_rng(s).standard_normal(s * n)
        lib.paradiag_capacitance_apply(plan, T(v), Jv)
        torch.cuda.synchronize()
        x, Jv = x.cpu().numpy(), Jv.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    assert np.linalg.norm(x - ref["x"].reshape(-1)) <= 1e-11 * np.linalg.norm(ref["x"])
    Jref = ref["J"] @ v
    assert np.linalg.norm(Jv - Jref) <= 1e-12 * np.linalg.norm(Jref)
    U, _ = _solve(lib, n, ell, tau, M, K, s, U0, F)
    assert allatonce.rel_err(U, ref["U"]) < 1e-11


@pytest.mark.parametrize("s", [2, 4, 6])
def test_bdf_forward_transform(lib, s):
    """Half spectrum of h (eq. discrete_probBDF without M) against numpy's FFT."""
    n, ell = 37, 32
    M, K, tau, U0, F = _problem("fem1", n, ell, s, s)
    Msp, _ = spatial_matrices(None, K, 1)           # identity: h itself
    h = bdf.rhs_bdf(Msp, tau, s, list(U0), F)
    ref = np.fft.fft(h, axis=0)[: ell // 2 + 1]
    plan = _plan(lib, n, ell, tau, M, K, s)
    try:
        Hhat = torch.empty((ell // 2 + 1, n), dtype=torch.complex128, device=dev())
        lib.paradiag_forward_transform(plan, T(U0), T(F), Hhat)
        torch.cuda.synchronize()
        got = Hhat.cpu().numpy()
        with pytest.raises(lib.PDError) as e:         # b is not the BDF b^(s)
            lib.paradiag_shifted_solve(plan, Hhat, None, None, torch.empty(n, dtype=torch.float64,
                                                                           device=dev()))
        assert e.value.status == lib.PD_ENOTSUP
    finally:
        lib.paradiag_plan_destroy(plan)
    assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)


@pytest.mark.parametrize("s", [2, 5])
def test_bdf_residual_entry(lib, s):
    n, ell = 31, 16
    M, K, tau, U0, F = _problem("fd1", n, ell, s, 3 + s)
    Msp, Ksp = spatial_matrices(M, K, 1)
    Uref = bdf.step_bdf(Msp, Ksp, tau, s, list(U0), F)
    Up = Uref + 1e-3 * np.random.default_rng(1).standard_normal(Uref.shape)
    G = bdf.rhs_bdf(Msp, tau, s, list(U0), F)
    expect = np.linalg.norm(G - bdf.apply_bdf(Msp, Ksp, tau, s, Up)) / np.linalg.norm(G)
    plan = _plan(lib, n, ell, tau, M, K, s)
    try:
        r0 = lib.paradiag_residual(plan, T(U0), T(F), T(Uref))
        r1 = lib.paradiag_residual(plan, T(U0), T(F), T(Up))
    finally:
        lib.paradiag_plan_destroy(plan)
    assert r0 < 1e-13
    assert abs(r1 - expect) <= 1e-10 * expect


@pytest.mark.parametrize("s", [2, 3, 6])
def test_bdf_full_size_exact(lib, s):
    """n = 8191, ell = 2048 FEM workload (sine-series data, all starting
    values equal to u0): U against the per-mode BDF recurrence."""
    p = wl.cfg_fem_1d()
    U0 = np.tile(p.u0, (s, 1))
    U, info = _solve(lib, p.n, p.ell, p.tau, p.M, p.K, s, U0, p.F, tol=1e-10)
    rng = np.random.default_rng(s)
    tt = rng.integers(0, p.ell, 4000)
    ii = rng.integers(0, p.n, 4000)
    ref = bdf.modal_bdf(p, s)
    err = np.linalg.norm(U[tt, ii] - ref[tt, ii]) / np.linalg.norm(ref[tt, ii])
    assert err < 1e-9, (err, info.as_dict())
    assert allatonce.rel_err(U, ref) < 1e-9
    assert info.pint_loops == info.gmres_iters + 2


def test_bdf_order1_is_backward_euler(lib):
    """bdf_order = 1 is the backward Euler plan itself (bitwise)."""
    p = wl.cfg_small_fd()
    outs = []
    for kw in ({}, {"bdf_order": 1}):
        plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, stream=_stream(), **kw)
        try:
            U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
            lib.paradiag_solve(plan, T(p.u0), T(p.F), U, 1e-10)
            torch.cuda.synchronize()
            outs.append(U.cpu().numpy())
        finally:
            lib.paradiag_plan_destroy(plan)
    assert np.array_equal(outs[0], outs[1])


def test_bdf_two_solves_in_a_row(lib):
    """A plan reused for a second right-hand side (the work buffers keep
    the first solve's contents) gives the second solution."""
    n, ell, s = 63, 32, 3
    M, K, tau, U0, F = _problem("fd1", n, ell, s, 11)
    _, _, _, U0b, Fb = _problem("fd1", n, ell, s, 12)
    Msp, Ksp = spatial_matrices(M, K, 1)
    plan = _plan(lib, n, ell, tau, M, K, s)
    try:
        U = torch.empty((ell, n), dtype=torch.float64, device=dev())
        lib.paradiag_solve(plan, T(U0), T(F), U, 1e-12)
        lib.paradiag_solve(plan, T(U0b), T(Fb), U, 1e-12)
        torch.cuda.synchronize()
        got = U.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    assert allatonce.rel_err(got, bdf.step_bdf(Msp, Ksp, tau, s, list(U0b), Fb)) < 1e-10


def test_bdf_rejects_unsupported(lib):
    p = wl.cfg_small_fd()
    bad = [dict(bdf_order=7), dict(bdf_order=0), dict(bdf_order=2, precision=lib.PD_MIXED),
           dict(bdf_order=2, alpha=0.5), dict(bdf_order=2, early_exit=1),
           dict(bdf_order=2, shifted_solver=lib.PD_SHIFTED_SINE)]
    for kw in bad:
        with pytest.raises(RuntimeError):
            lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, **kw)
    with pytest.raises(RuntimeError):            # ell < 2 s
        lib.paradiag_plan_create(p.n, 8, p.tau, p.M, p.K, bdf_order=5)


# ------------------------------------------------ block Galerkin for J^(s) --

def _bg_problem(kind, n, ell, T_, s):
    p = wl.heat_1d(kind, n, ell, T_, 1.0, np.random.default_rng(n + ell), True)
    return p, np.tile(p.u0, (s, 1))


def _bg_solve(lib, p, U0, s, tol, **kw):
    plan = _plan(lib, p.n, p.ell, p.tau, p.M, p.K, s, krylov=lib.PD_KRYLOV_FOM,
                 check_residual=1, **kw)
    try:
        U = torch.empty((p.ell, p.n), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(U0), T(p.F), U, tol, allow_notconv=True)
        torch.cuda.synchronize()
        return U.cpu().numpy(), info
    finally:
        lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("kind,n,ell,T_,s", [
    ("fd1", 15, 16, 1.0, 3), ("fd1", 31, 16, 1.0, 2), ("fd1", 31, 16, 1.0, 6),
    ("fem1", 31, 16, 1.0, 3), ("fd1", 127, 16, 4.0, 3), ("fem1", 511, 32, 10.0, 2),
    ("fem1", 511, 32, 10.0, 3), ("fd1", 9, 16, 1.0, 3), ("fem1", 4, 8, 1.0, 2)])
def test_block_galerkin_matches_oracle(lib, kind, n, ell, T_, s):
    """Same number of block steps as the oracle's block Galerkin method at
    the same tolerance (tol/100 on ||r|| / ||b||; one step either way at the
    threshold), #PinT = checks + 2, and the same U."""
    p, U0 = _bg_problem(kind, n, ell, T_, s)
    tol = 1e-10
    U, info = _bg_solve(lib, p, U0, s, tol)
    Msp, Ksp = problem_matrices(p)
    ref = bdf.paradiag_bdf(Msp, Ksp, p.tau, s, list(U0), p.F, capacitance="galerkin",
                           eps=tol * 1e-2, maxit=32 // s)
    assert ref["history"][-1] <= tol * 1e-2 * np.linalg.norm(ref["b"])
    assert abs(info.gmres_iters - ref["steps"]) <= 1, (info.as_dict(), ref["steps"])
    assert info.pint_loops == info.gmres_iters + 2
    assert allatonce.rel_err(U, ref["U"]) < 1e-10
    D = bdf.step_bdf(Msp, Ksp, p.tau, s, list(U0), p.F)
    assert allatonce.rel_err(U, D) < 1e-10
    assert 0 <= info.rel_residual < 1e-9


def test_block_galerkin_residual_matches_oracle(lib):
    """The residual norm after m = 1, 2, 3 block steps (maxit = m) equals
    the oracle's ||(I - I_s (x) V V^T) S y|| there (residuals well above
    rounding: after 10 steps it is 1.5e-11 ||b|| and rounding moves it by
    a few per cent on either side)."""
    p, U0 = _bg_problem("fem1", 255, 16, 10.0, 3)
    Msp, Ksp = problem_matrices(p)
    ref = bdf.paradiag_bdf(Msp, Ksp, p.tau, 3, list(U0), p.F, capacitance="galerkin",
                           eps=0.0, maxit=3)
    for m in (1, 2, 3):
        U, info = _bg_solve(lib, p, U0, 3, 1e-10, maxit=m)
        assert info.gmres_iters == m
        rel = ref["history"][m - 1] / np.linalg.norm(ref["b"])
        assert abs(info.gmres_rel_residual - rel) <= 1e-5 * rel, (m, info.gmres_rel_residual, rel)


@pytest.mark.parametrize("q", [2, 3])
def test_block_galerkin_residual_freezing(lib, q):
    p, U0 = _bg_problem("fd1", 31, 16, 1.0, 3)
    U, info = _bg_solve(lib, p, U0, 3, 1e-10, fom_q=q)
    assert info.gmres_iters % q == 0 or info.gmres_iters == 32 // 3
    assert info.pint_loops == -(-info.gmres_iters // q) + 2
    Msp, Ksp = problem_matrices(p)
    D = bdf.step_bdf(Msp, Ksp, p.tau, 3, list(U0), p.F)
    assert allatonce.rel_err(U, D) < 1e-10


def test_block_galerkin_step_cap_is_reported(lib):
    p, U0 = _bg_problem("fem1", 255, 16, 10.0, 3)
    plan = _plan(lib, p.n, p.ell, p.tau, p.M, p.K, 3, krylov=lib.PD_KRYLOV_FOM)
    try:
        U = torch.empty((p.ell, p.n), dtype=torch.float64, device=dev())
        with pytest.raises(lib.PDError) as e:
            lib.paradiag_solve(plan, T(U0), T(p.F), U, 1e-12)
        assert e.value.status == lib.PD_ENOTCONV
    finally:
        lib.paradiag_plan_destroy(plan)


def test_block_galerkin_zero_data_and_small_n(lib):
    """Zero data gives x = 0 and U = 0 without building a block space; a
    block Galerkin plan needs n >= s."""
    n, ell, s = 31, 16, 3
    M, K = wl.fem_mass(n), wl.fem_stiffness(n, 1.0)
    plan = _plan(lib, n, ell, 1.0 / ell, M, K, s, krylov=lib.PD_KRYLOV_FOM)
    try:
        U = torch.full((ell, n), 7.0, dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(np.zeros((s, n))), T(np.zeros((ell, n))), U, 1e-10)
        torch.cuda.synchronize()
        assert info.gmres_iters == 0
        assert not U.cpu().numpy().any()
    finally:
        lib.paradiag_plan_destroy(plan)
    with pytest.raises(RuntimeError):
        _plan(lib, 3, 16, 1.0 / 16, None, wl.fd_laplacian(3, 1.0), 4, krylov=lib.PD_KRYLOV_FOM)


# ------------------------------------------------------------------- 2D --

# n = 10 and 20: the chirp-z DST along x (n + 1 not a power of two)
@pytest.mark.parametrize("n,ell,s", [(15, 16, 2), (31, 32, 3), (15, 16, 6), (63, 16, 4),
                                     (10, 16, 2), (20, 16, 3)])
def test_bdf_2d_matches_stepping(lib, n, ell, s):
    """2D FD heat (M = I, K = I (x) T + T (x) I; the DST-x domain of the
    shifted solves): random starting values and source, U against BDF
    stepping with the 2D sparse matrices, and the reported residual."""
    rng = np.random.default_rng(17 * n + s)
    p = wl.heat_2d(n, ell, 0.1, 1.0, rng)
    U0 = rng.standard_normal((s, p.nbar))
    F = rng.standard_normal((ell, p.nbar))
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, None, p.K, dims=2, bdf_order=s,
                                    check_residual=1, stream=_stream())
    try:
        U = torch.empty((ell, p.nbar), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(U0), T(F), U, 1e-12)
        r = lib.paradiag_residual(plan, T(U0), T(F), U)
        torch.cuda.synchronize()
        got = U.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    Msp, Ksp = problem_matrices(p)
    ref = bdf.step_bdf(Msp, Ksp, p.tau, s, list(U0), F)
    err = allatonce.rel_err(got, ref)
    assert err < 1e-10, (err, info.as_dict())
    assert info.pint_loops == info.gmres_iters + 2
    G = bdf.rhs_bdf(Msp, p.tau, s, list(U0), F)
    res = np.linalg.norm(G - bdf.apply_bdf(Msp, Ksp, p.tau, s, got)) / np.linalg.norm(G)
    assert abs(r - res) <= 1e-6 * res + 1e-15 and r < 1e-10
    assert abs(info.rel_residual - r) <= 1e-12


@pytest.mark.parametrize("n", [7, 6])
def test_bdf_2d_capacitance_apply(lib, n):
    """The 2D block product against the oracle's dense J^(s) (n = 6: the
    chirp-z DST along x)."""
    ell, s = 16, 2
    rng = np.random.default_rng(3)
    p = wl.heat_2d(n, ell, 0.1, 1.0, rng)
    U0 = rng.standard_normal((s, p.nbar))
    F = rng.standard_normal((ell, p.nbar))
    Msp, Ksp = problem_matrices(p)
    ref = bdf.paradiag_bdf(Msp, Ksp, p.tau, s, list(U0), F)
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, None, p.K, dims=2, bdf_order=s,
                                    stream=_stream())
    try:
        v = rng.standard_normal(s * p.nbar)
        Jv = torch.empty(s * p.nbar, dtype=torch.float64, device=dev())
        lib.paradiag_capacitance_apply(plan, T(v), Jv)
        torch.cuda.synchronize()
        got = Jv.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    want = ref["J"] @ v
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


@pytest.mark.parametrize("n,ell,T_,s", [(15, 16, 1.0, 2), (15, 16, 1.0, 3), (31, 16, 1.0, 2),
                                        (20, 16, 1.0, 2)])
def test_bdf_2d_block_galerkin_matches_oracle(lib, n, ell, T_, s):
    """The block Galerkin method on 2D plans (in the DST-x domain, multi-block
    Gram-Schmidt): the oracle's step count and U."""
    p = wl.heat_2d(n, ell, T_, 1.0, np.random.default_rng(n + ell))
    U0 = np.tile(p.u0, (s, 1))
    tol = 1e-10
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, None, p.K, dims=2, bdf_order=s,
                                    krylov=lib.PD_KRYLOV_FOM, check_residual=1,
                                    stream=_stream())
    try:
        U = torch.empty((ell, p.nbar), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(U0), T(p.F), U, tol)
        torch.cuda.synchronize()
        got = U.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    Msp, Ksp = problem_matrices(p)
    ref = bdf.paradiag_bdf(Msp, Ksp, p.tau, s, list(U0), p.F, capacitance="galerkin",
                           eps=tol * 1e-2, maxit=32 // s)
    assert abs(info.gmres_iters - ref["steps"]) <= 1, (info.as_dict(), ref["steps"])
    assert info.pint_loops == info.gmres_iters + 2
    assert allatonce.rel_err(got, ref["U"]) < 1e-10
    assert 0 <= info.rel_residual < 1e-10


@pytest.mark.parametrize("s", [2, 3])
def test_bdf_2d_full_size_sampled(lib, s):
    """511 x 511 grid, ell = 256, T = 0.1 (the 2D FD workload), every
    starting value u0: sampled outputs against the per-mode BDF recurrence."""
    p = wl.cfg_fd_2d()
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, None, p.K, dims=2, bdf_order=s,
                                    stream=_stream())
    try:
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(np.tile(p.u0, (s, 1))), T(p.F), U, 1e-10)
        torch.cuda.synchronize()
        rng = np.random.default_rng(s)
        tt = rng.integers(0, p.ell, 4000)
        ii = rng.integers(0, p.nbar, 4000)
        got = U[torch.tensor(tt, device=dev()), torch.tensor(ii, device=dev())].cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    ref = bdf.modal_bdf(p, s, (tt, ii))
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-9, (err, info.as_dict())
