"""Error paths of the C ABI on the GPU: a singular zero-frequency block, a
non-finite input, and a capacitance solve that cannot reach its tolerance
(PD_ENOTCONV with the last iterate in U)."""
import numpy as np
import pytest

from oracle import allatonce, modal
from paper_2304_12597_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=dev())


def stream():
    return torch.cuda.current_stream().cuda_stream


def neumann_stiffness(n, nu=1.0):
    """nu tridiag(-1, 2, -1) / h^2 with the first and last diagonal entries
    set to nu / h^2: every row sums to zero, so K (and tau K) is singular."""
    lower, diag, upper = wl.fd_laplacian(n, nu)
    diag = diag.copy()
    diag[0] = diag[-1] = 0.5 * diag[1]
    return lower, diag, upper


@pytest.mark.parametrize("kind", ["fd1", "fem1"])
def test_singular_zero_frequency_block(lib, kind):
    """alpha = 1: P_0 = tau K is the zero-frequency block (Section 2), so a
    pure-Neumann K is rejected with PD_ESINGULAR; with alpha < 1 (Section 4)
    no shift is zero and the plan is accepted."""
    n, ell = 63, 16
    h = 1.0 / (n + 1)
    K = neumann_stiffness(n)
    M = None
    if kind == "fem1":
        K = tuple(a * h for a in K)      # the same pattern with the FEM scaling nu / h
        M = wl.fem_mass(n)
    with pytest.raises(lib.PDError) as ei:
        lib.paradiag_plan_create(n, ell, 1.0 / ell, M, K, stream=stream())
    assert ei.value.status == lib.PD_ESINGULAR
    plan = lib.paradiag_plan_create(n, ell, 1.0 / ell, M, K, alpha=0.5, stream=stream())
    lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("where", ["u0", "F"])
@pytest.mark.parametrize("prec,dims", [(0, 1), (1, 1), (0, 2), (2, 1)])
def test_nonfinite_input(lib, where, prec, dims):
    """A NaN in u0 or in F makes the capacitance right-hand side b
    non-finite; the solve returns PD_ENONFINITE instead of a result."""
    rng = np.random.default_rng(5)
    if dims == 1:
        p = wl.heat_1d("fem1", 255, 32, 1.0, 1.0, rng, True)
    else:
        p = wl.heat_2d(31, 16, 0.1, 1.0, rng)
    u0, F = p.u0.copy(), p.F.copy()
    if where == "u0":
        u0[17] = np.nan
    else:
        F[3, 11] = np.nan
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, dims=dims, precision=prec,
                                    stream=stream())
    try:
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        with pytest.raises(lib.PDError) as ei:
            lib.paradiag_solve(plan, T(u0), T(F), U, 1e-8)
        assert ei.value.status == lib.PD_ENONFINITE, ei.value
        # the plan stays usable: the same problem with finite data solves
        info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, 1e-8 if prec != 2 else 1e-5)
        torch.cuda.synchronize()
        err = allatonce.rel_err(U.cpu().numpy(), modal.modal_solution(p))
        assert err < (1e-8 if prec != 2 else 1e-3), (err, info.as_dict())
    finally:
        lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("prec", [0, 1])
def test_capacitance_not_converged_returns_last_iterate(lib, prec):
    """With the capacitance GMRES capped at one iteration and a tolerance it
    cannot reach, the solve returns PD_ENOTCONV and U holds the result of
    the last iterate (here an ill-conditioned J: nu = 1e-3).  In float64,
    U is the all-at-once solution built from x_1, the oracle's one-step
    GMRES iterate: the second parfor with x is the circulant solve of G with
    g_1 replaced by g_1 - M x (Section 2), i.e. the alpha-circulant solution
    for the initial value u0 - x.  In mixed precision U is finite and closer
    to the solution than the uncorrected first term."""
    from oracle import paradiag
    from oracle.spatial import problem_matrices
    p = wl.heat_1d("fd1", 1000, 128, 1.0, 1e-3, np.random.default_rng(8), True)
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, precision=prec, maxit=1,
                                    max_sweeps=2, stream=stream())
    try:
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        with pytest.raises(lib.PDError) as ei:
            lib.paradiag_solve(plan, T(p.u0), T(p.F), U, 1e-14)
        assert ei.value.status == lib.PD_ENOTCONV
        info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, 1e-14, allow_notconv=True)
        torch.cuda.synchronize()
        Ug = U.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    assert np.isfinite(Ug).all()
    assert info.gmres_iters >= 1 and 1e-16 < info.gmres_rel_residual < 1.0
    Msp, Ksp = problem_matrices(p)
    U1 = paradiag.periodic_solution(Msp, Ksp, p.tau, p.u0, p.F)
    Uref = modal.modal_solution(p)
    if prec == 0:
        cap = paradiag.Capacitance(Msp, Ksp, p.tau, p.ell)
        b = paradiag.capacitance_rhs(U1)
        x1, its, _ = paradiag.gmres(lambda v: cap.matvec(v).real, b, tol=1e-30, maxit=1)
        assert its == 1
        Ux1 = paradiag.periodic_solution(Msp, Ksp, p.tau, p.u0 - np.real(x1), p.F)
        assert allatonce.rel_err(Ug, Ux1) < 1e-9, allatonce.rel_err(Ug, Ux1)
        assert allatonce.rel_err(Ux1, Uref) > 1e-6      # x_1 is not the solution
    else:
        assert allatonce.rel_err(Ug, Uref) < allatonce.rel_err(U1, Uref)
