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


def _mixed_run(lib, p, max_sweeps, tol, dims=1):
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, precision=1, dims=dims,
                                    max_sweeps=max_sweeps, stream=stream())
    try:
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        status, msg = lib.PD_OK, ""
        try:
            info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, tol)
        except lib.PDError as e:
            assert e.status == lib.PD_ENOTCONV, e
            status, msg = e.status, lib.paradiag_last_error()
            info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, tol, allow_notconv=True)
        torch.cuda.synchronize()
        return U.cpu().numpy(), info, status, msg
    finally:
        lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("case", ["fem1-stiff", "fd1-floor", "fd2-floor"])
def test_mixed_refinement_stall_returns_best_iterate(lib, case):
    """PD_MIXED refinement stops when a sweep no longer lowers the float64
    all-at-once residual: it takes that sweep's correction back and returns
    PD_ENOTCONV with the best iterate, before max_sweeps.  The returned U's
    residual (oracle, CPU) is the smallest over the iterates, which runs
    capped at k = 1, 2, ... sweeps reproduce, and info.rel_residual is it.
    Cases: a stiff FEM problem (tau mu_max ~ 2e8, where float32 elimination
    barely contracts) at a reachable-looking tolerance, and tolerances below
    the float64 residual floor in 1D and 2D."""
    from oracle.spatial import problem_matrices
    rng = np.random.default_rng(11)
    if case == "fem1-stiff":
        p, dims, tol = wl.heat_1d("fem1", 16383, 16, 1.0, 1.0, rng, True), 1, 1e-10
    elif case == "fd1-floor":
        p, dims, tol = wl.heat_1d("fd1", 1023, 64, 1.0, 1.0, rng, True), 1, 1e-17
    else:
        p, dims, tol = wl.heat_2d(31, 16, 0.1, 1.0, rng), 2, 1e-17
    print("stall case", case, p.n, p.ell, flush=True)
    max_sweeps = 16
    U, info, status, msg = _mixed_run(lib, p, max_sweeps, tol, dims)
    assert np.isfinite(U).all()
    Msp, Ksp = problem_matrices(p)
    res = lambda V: allatonce.residual(Msp, Ksp, p.tau, p.u0, p.F, V)[1]
    r = res(U)
    # rounding floor of a computed relative residual: a few units of float64
    # roundoff times || |A| |U| + |G| || / ||G|| (|A| the entrywise absolute
    # all-at-once operator); on the stiff problem it is above 1e-9
    G = allatonce.rhs(Msp, p.tau, p.u0, p.F)
    aU = np.abs(U)
    AU = np.asarray((abs(Msp + p.tau * Ksp) @ aU.T).T)
    AU[1:] += np.asarray((abs(Msp) @ aU[:-1].T).T)
    floor = 8 * 2.0 ** -53 * np.linalg.norm(AU + np.abs(G)) / np.linalg.norm(G)
    if status == lib.PD_OK:                  # converged after all
        assert info.rel_residual <= tol and r <= 10 * tol
        return
    assert "stalled" in msg, msg
    assert 2 <= info.sweeps < max_sweeps, info.as_dict()
    # the iterates after k = 1 .. sweeps - 1 sweeps (the last sweep was taken back)
    rk = [res(_mixed_run(lib, p, k, tol, dims)[0]) for k in range(1, info.sweeps)]
    best = min(rk)
    assert r <= 1.5 * best + floor, (r, rk, floor)
    assert abs(info.rel_residual - r) <= 0.5 * r + floor, (info.rel_residual, r, floor)
