"""GPU parity: every stage of the HIP path, called through the C ABI, against
the CPU oracle on the same seeded inputs (element by element)."""
import numpy as np
import pytest

from oracle import allatonce, modal, paradiag
from oracle.spatial import problem_matrices, spatial_matrices
from paper_2304_12597_amd import workloads as wl

from bounds import fp64_error_bound, tau_mu_range

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=dev())


def cplx_view(t, dtype):
    """Interleaved complex buffer -> numpy complex array."""
    a = t.cpu().numpy()
    return a.view(dtype)


def make_problem(kind, n, ell, seed, nu=1.0, T_=1.0, with_source=True):
    return wl.heat_1d(kind, n, ell, T_, nu, np.random.default_rng(seed), with_source)


def plan_for(lib, p, **kw):
    return lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K,
                                    stream=torch.cuda.current_stream().cuda_stream, **kw)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


PRECS = {"fp64": (0, np.complex128, torch.float64, 1e-12),
         "fp32": (2, np.complex64, torch.float32, 2e-5)}


# ------------------------------------------------------------ transforms --

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ell", [(2, 2), (5, 4), (37, 8), (63, 32), (101, 256),
                                   (33, 2048), (9, 4096), (1000, 64)])
@pytest.mark.parametrize("alpha", [1.0, 0.01])
def test_forward_transform(lib, prec, n, ell, alpha):
    code, cdt, rdt, tol = PRECS[prec]
    p = make_problem("fd1", n, ell, n + ell)
    rng = np.random.default_rng(ell)
    p.u0 = rng.standard_normal(n)
    p.F = rng.standard_normal((ell, n))
    plan = plan_for(lib, p, precision=code, alpha=alpha)
    try:
        nb = lib.paradiag_spectrum_bytes(plan)
        F2 = ell // 2 + 1
        assert nb == F2 * n * np.dtype(cdt).itemsize
        H = torch.empty(nb // (8 if prec == "fp64" else 4), dtype=rdt, device=dev())
        lib.paradiag_forward_transform(plan, T(p.u0), T(p.F), H)
        torch.cuda.synchronize()
        got = cplx_view(H, cdt).reshape(F2, n)
    finally:
        lib.paradiag_plan_destroy(plan)
    Hrows = allatonce.rhs(spatial_matrices(None, p.K, 1)[0], p.tau, p.u0, p.F)
    w = alpha ** (1.0 / ell)
    ref = np.fft.fft((w ** np.arange(ell))[:, None] * Hrows, axis=0)[:F2]
    assert rel(got, ref) < tol, rel(got, ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,ell", [(2, 2), (37, 8), (63, 32), (101, 256), (33, 2048),
                                   (9, 4096), (1000, 64)])
def test_inverse_transform(lib, prec, n, ell):
    code, cdt, rdt, tol = PRECS[prec]
    p = make_problem("fd1", n, ell, 3)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((ell, n))
    F2 = ell // 2 + 1
    spec = np.ascontiguousarray(np.fft.fft(X, axis=0)[:F2]).astype(cdt)
    plan = plan_for(lib, p, precision=code)
    try:
        Sbuf = torch.tensor(spec.view(np.float64 if prec == "fp64" else np.float32).reshape(-1),
                            device=dev())
        U = torch.empty((ell, n), dtype=torch.float64, device=dev())
        lib.paradiag_inverse_transform(plan, Sbuf, U)
        torch.cuda.synchronize()
        got = U.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    assert rel(got, X) < tol * 4, rel(got, X)


# ---------------------------------------------------------- shifted solves --

def _oracle_pieces(p, alpha=1.0):
    """The oracle's pieces, each from its own definition: b (a time slice of
    the alpha-circulant solution U_1, by stepping), x = J^{-1} b (dense J),
    and Y_k = P_k^{-1} (Ghat_k - w M x) for every frequency; Hhat is the
    spectrum without the mass matrix (what the GPU's forward transform
    produces)."""
    Msp, Ksp = problem_matrices(p)
    cap = paradiag.Capacitance(Msp, Ksp, p.tau, p.ell, alpha)
    U1 = paradiag.periodic_solution(Msp, Ksp, p.tau, p.u0, p.F, alpha)
    b = paradiag.capacitance_rhs(U1, alpha)
    x = paradiag.capacitance_solution(cap, b, "dense")
    w = alpha ** (1.0 / p.ell)
    Ghat = paradiag.rhs_spectrum(Msp, p.tau, p.u0, p.F, alpha)
    Y = paradiag.shifted_solutions(cap, Ghat - w * (Msp @ x)[None, :])
    Hrows = allatonce.rhs(spatial_matrices(None, p.K, 1)[0], p.tau, p.u0, p.F)
    Hhat = np.fft.fft((w ** np.arange(p.ell))[:, None] * Hrows, axis=0)
    return dict(pi=cap.pi, b=b, x=x, Y=Y), Hhat


SOLVE_CASES = [("fd1", 7, 8), ("fem1", 63, 32), ("fem1", 100, 16), ("fd1", 257, 64),
               ("fem1", 1000, 8), ("fd1", 2, 4), ("fd1", 3, 2), ("fem1", 4097, 4)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("kind,n,ell", SOLVE_CASES)
@pytest.mark.parametrize("alpha", [1.0, 0.05])
def test_shifted_solves_and_b(lib, prec, kind, n, ell, alpha):
    code, cdt, rdt, tol = PRECS[prec]
    # complex64 forward error grows with the condition number of P_k (about
    # (n+1)^2); above n = 300 the solves are checked by their backward error
    backward_only = prec == "fp32" and n > 300
    p = make_problem(kind, n, ell, n * 7 + ell, nu=0.3)
    out, Hhat = _oracle_pieces(p, alpha)
    F2 = ell // 2 + 1
    w = alpha ** (1.0 / ell)
    plan = plan_for(lib, p, precision=code, alpha=alpha)
    try:
        Hbuf = torch.tensor(np.ascontiguousarray(Hhat[:F2]).astype(cdt).view(
            np.float64 if prec == "fp64" else np.float32).reshape(-1), device=dev())
        Y = torch.empty_like(Hbuf)
        b = torch.empty(n, dtype=torch.float64, device=dev())
        x = T(out["x"])
        lib.paradiag_shifted_solve(plan, Hbuf, x, Y, b)
        torch.cuda.synchronize()
        Yg = cplx_view(Y, cdt).reshape(F2, n)
        bg = b.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    if backward_only:
        # P_k Y_k = M (Hhat_k - w x) for every k, up to a normwise backward
        # error of a few float32 units (the complex64 rounding of the oracle's
        # own Y gives 2e-8 here; dropping w x gives 3e-6, a conjugated Y, two
        # frequencies swapped or one row off by 1e-3 give 1.6e-5 to 2.5e-5)
        Msp, Ksp = problem_matrices(p)
        Mcsr = Msp.tocsr()
        for k in range(F2):
            Pk = ((1.0 - out["pi"][k]) * Msp + p.tau * Ksp).tocsr()
            rhs = Mcsr @ (Hhat[k] - w * out["x"])
            Yk = Yg[k].astype(np.complex128)
            r = Pk @ Yk - rhs
            nP = float(abs(Pk).sum(axis=1).max())
            be = np.linalg.norm(r) / (nP * np.linalg.norm(Yk) + np.linalg.norm(rhs))
            print("k=%d backward error %.2e" % (k, be))
            assert be < 2e-7, (k, be)
        assert np.isfinite(bg).all()
        return
    # Y_k = L_k - w W_k (second parfor), b = L F^{-T} e_ell (first parfor)
    Yref = out["Y"][:F2]
    tolY = 1e-10 if prec == "fp64" else 2e-3
    assert rel(Yg, Yref) < tolY, rel(Yg, Yref)
    # b sums ell solutions of systems with condition number ~ (n+1)^2, and
    # the oracle's b comes from a different algorithm (the alpha-circulant
    # solution by stepping); two correct algorithms differ by ~ cond * eps,
    # times the condition alpha^(-(ell-1)/ell) of the scaled DFT
    kappa_alpha = alpha ** (-(ell - 1) / ell)
    assert rel(bg, out["b"]) < (max(1e-10, 1e-16 * (n + 1) ** 2) * kappa_alpha
                                if prec == "fp64" else 2e-3)


@pytest.mark.parametrize("kind,n,ell", SOLVE_CASES[:6])
def test_capacitance_apply_and_solve(lib, kind, n, ell):
    p = make_problem(kind, n, ell, 11, nu=0.05)
    Msp, Ksp = problem_matrices(p)
    cap = paradiag.Capacitance(Msp, Ksp, p.tau, ell)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(n)
    Jv_ref = cap.matvec(v)
    assert np.max(np.abs(Jv_ref.imag)) < 1e-10 * np.max(np.abs(Jv_ref))
    plan = plan_for(lib, p, precision=0)
    try:
        Jv = torch.empty(n, dtype=torch.float64, device=dev())
        lib.paradiag_capacitance_apply(plan, T(v), Jv)
        x = torch.empty(n, dtype=torch.float64, device=dev())
        its, rr = lib.paradiag_capacitance_solve(plan, T(v), x, 1e-12)
        torch.cuda.synchronize()
        Jg, xg = Jv.cpu().numpy(), x.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    assert rel(Jg, Jv_ref.real) < 1e-12
    xref = np.linalg.solve(cap.dense(), v).real
    assert rel(xg, xref) < 1e-10, rel(xg, xref)
    assert rr <= 1e-12 and its >= 1


# ------------------------------------------------------------- end to end --

def _solve(lib, p, prec=0, tol=1e-10, **kw):
    plan = plan_for(lib, p, precision=prec, check_residual=1, **kw)
    try:
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, tol)
        torch.cuda.synchronize()
        return U.cpu().numpy(), info
    finally:
        lib.paradiag_plan_destroy(plan)


def test_small_fd_config_fp64(lib):
    p = wl.cfg_small_fd()
    U, info = _solve(lib, p)
    assert allatonce.rel_err(U, modal.modal_solution(p)) < 1e-10
    assert allatonce.rel_err(U, allatonce.step(p)) < 1e-10
    assert 0 <= info.rel_residual < 1e-12
    assert info.pint_loops == info.gmres_iters + 2


def test_small_fd_config_mixed_and_fp32(lib):
    p = wl.cfg_small_fd()
    Uref = modal.modal_solution(p)
    U, info = _solve(lib, p, prec=1, tol=1e-10)
    assert allatonce.rel_err(U, Uref) < 1e-8, (allatonce.rel_err(U, Uref), info.as_dict())
    assert info.sweeps >= 2 and info.rel_residual <= 1e-10
    U32, info32 = _solve(lib, p, prec=2, tol=1e-6)
    assert allatonce.rel_err(U32, Uref) < 1e-4


@pytest.mark.parametrize("kind,n,ell,nu", [
    ("fd1", 2, 2, 1.0), ("fd1", 3, 4, 1.0), ("fem1", 5, 8, 0.1), ("fd1", 100, 16, 0.01),
    ("fem1", 255, 64, 1.0), ("fd1", 1000, 128, 0.001), ("fem1", 4095, 256, 1.0),
    ("fd1", 8191, 32, 1.0), ("fem1", 1023, 2048, 0.001), ("fd1", 63, 4096, 1.0)])
def test_end_to_end_fp64(lib, kind, n, ell, nu):
    p = make_problem(kind, n, ell, n + 3 * ell, nu=nu)
    U, info = _solve(lib, p)
    Uref = modal.modal_solution(p)
    err = allatonce.rel_err(U, Uref)
    bound = fp64_error_bound(p, 1e-10)
    stiff = tau_mu_range(p)[1]
    print("%s n=%d ell=%d nu=%g tau*mu_max=%.2e err=%.3e bound=%.1e res=%.3e gmres=%d" % (
        kind, n, ell, nu, stiff, err, bound, info.rel_residual, info.gmres_iters))
    assert err < bound, (err, bound, info.as_dict())
    # the float64 residual of a direct shifted solve sits at about u times
    # the problem's stiffness (1.8e-10 at tau mu_max = 7.9e5, 1.0e-9 at
    # 8.4e6): bounded by 4u tau mu_max, and 1e-10 for the mild cases
    assert 0 <= info.rel_residual < max(1e-10, 2.0 ** -51 * stiff)


@pytest.mark.parametrize("alpha", [0.5, 1e-2])
def test_end_to_end_alpha(lib, alpha):
    p = make_problem("fem1", 31, 16, 5, nu=0.01)
    U, info = _solve(lib, p, alpha=alpha)
    Msp, Ksp = problem_matrices(p)
    U2 = allatonce.solve_dense(Msp, Ksp, p.tau, p.u0, p.F)
    assert allatonce.rel_err(U, U2) < 1e-9


def _first_term_ratio(p, alpha):
    """Oracle: U_1 of Algorithm 3 and ||G - A(U_1)||_F / ||M U_1||_F."""
    Msp, Ksp = problem_matrices(p)
    U1 = paradiag.periodic_solution(Msp, Ksp, p.tau, p.u0, p.F, alpha)
    R, _ = allatonce.residual(Msp, Ksp, p.tau, p.u0, p.F, U1)
    MU1 = np.asarray((Msp @ U1.T).T)
    return U1, float(np.linalg.norm(R) / np.linalg.norm(MU1))


# alpha large enough that the exact first-term residual (alpha M u_ell)
# dominates the rounding residual ||A|| kappa u of the computed U_1
@pytest.mark.parametrize("kind,n,ell,alpha", [("fd1", 63, 32, 1e-2), ("fem1", 255, 64, 1e-2),
                                               ("fd1", 1000, 256, 0.1)])
def test_alpha_early_exit(lib, kind, n, ell, alpha):
    """Algorithm 3's test on the first term: with tol just above the oracle's
    residual ratio of U_1 the solve returns U_1 (one parfor, no capacitance
    solve); just below it, the full method runs and U solves the original
    system."""
    p = make_problem(kind, n, ell, 7 + n, nu=0.1)
    U1, ratio = _first_term_ratio(p, alpha)
    kappa = alpha ** (-(ell - 1) / ell)   # condition of the scaled DFT
    U, info = _solve(lib, p, tol=1.05 * ratio, alpha=alpha, early_exit=1)
    assert info.early_exit == 1 and info.gmres_iters == 0 and info.pint_loops == 1
    # the float64 bar, widened by the condition of the scaled DFT
    assert allatonce.rel_err(U, U1) < 1e-10 * max(1.0, kappa / 100), allatonce.rel_err(U, U1)
    tol = 0.95 * ratio
    U, info = _solve(lib, p, tol=tol, alpha=alpha, early_exit=1)
    assert info.early_exit == 0 and info.gmres_iters >= 1
    # the full method to the requested tolerance (GMRES stops at tol/100 ||b||)
    Uref = modal.modal_solution(p)
    assert allatonce.rel_err(U, Uref) < tol, allatonce.rel_err(U, Uref)
    assert 0 <= info.rel_residual < tol


def test_alpha_early_exit_2d(lib):
    p = wl.heat_2d(31, 16, 0.1, 1.0, np.random.default_rng(3))
    alpha = 1e-2
    U1, ratio = _first_term_ratio(p, alpha)
    U, info = _solve(lib, p, tol=1.05 * ratio, alpha=alpha, early_exit=1, dims=2)
    assert info.early_exit == 1 and info.gmres_iters == 0
    assert allatonce.rel_err(U, U1) < 1e-10
    tol = 0.95 * ratio
    U, info = _solve(lib, p, tol=tol, alpha=alpha, early_exit=1, dims=2)
    assert info.early_exit == 0
    assert allatonce.rel_err(U, allatonce.step(p)) < tol
    assert 0 <= info.rel_residual < tol


def test_end_to_end_nonuniform_matrices(lib):
    """General (non-constant-diagonal) SPD M and K use the per-row kernel."""
    n, ell = 77, 16
    rng = np.random.default_rng(4)
    kd = 2.0 + rng.uniform(0, 1, n); ko = -rng.uniform(0.2, 0.9, n)
    md = 4.0 + rng.uniform(0, 1, n); mo = rng.uniform(0.2, 0.9, n)
    K = (np.r_[0.0, ko[1:]], kd * 50, np.r_[ko[1:], 0.0])
    K = (K[0] * 50, K[1], K[2] * 50)
    M = (np.r_[0.0, mo[1:]], md, np.r_[mo[1:], 0.0])
    u0 = rng.standard_normal(n)
    F = rng.standard_normal((ell, n))
    p = wl.HeatProblem("fem1", n, ell, 1.0, 1.0, M, K, u0, F)
    U, info = _solve(lib, p)
    Msp, Ksp = problem_matrices(p)
    U1 = allatonce.step_1d(M, K, p.tau, u0, F)
    assert allatonce.rel_err(U, U1) < 1e-10


def test_fem_full_size_sampled(lib):
    """n = 8191, ell = 2048 FEM workload in the float64 form, on sampled
    outputs of the exact modal solution and the float64 residual."""
    p = wl.cfg_fem_1d()
    U, info = _solve(lib, p, tol=1e-8)
    rng = np.random.default_rng(0)
    tt = rng.integers(0, p.ell, 4000)
    ii = rng.integers(0, p.n, 4000)
    ref = modal.modal_sample(p, tt, ii)
    err = np.linalg.norm(U[tt, ii] - ref) / np.linalg.norm(ref)
    assert err < 1e-8, (err, info.as_dict())
    assert 0.0 <= info.rel_residual < 1e-8
    assert np.allclose(U[-1, ii[:50]], modal.modal_sample(p, np.full(50, p.ell - 1), ii[:50]),
                       rtol=1e-6, atol=1e-9)


def _sampled_err(p, U, seed=0, count=4000):
    rng = np.random.default_rng(seed)
    tt = rng.integers(0, p.ell, count)
    ii = rng.integers(0, p.nbar, count)
    tt[:2] = [0, p.ell - 1]
    ii[:2] = [0, p.nbar - 1]
    ref = modal.modal_sample(p, tt, ii)
    return float(np.linalg.norm(U[tt, ii] - ref) / np.linalg.norm(ref))


def test_fem_full_size_mixed_sampled(lib):
    """n = 8191, ell = 2048 FEM workload in the mixed form (complex64
    transforms and shifted solves, float64 residual refinement): PD_OK, the
    float64 residual at most tol, and the error against the exact modal
    solution at most 1e-8 on sampled outputs."""
    p = wl.cfg_fem_1d()
    U, info = _solve(lib, p, prec=1, tol=1e-8)      # raises unless PD_OK
    err = _sampled_err(p, U)
    print("fem1d mixed: err=%.3e res=%.3e sweeps=%d gmres=%d" % (
        err, info.rel_residual, info.sweeps, info.gmres_iters))
    assert err < 1e-8, (err, info.as_dict())
    assert 0.0 <= info.rel_residual <= 1e-8
    assert info.sweeps >= 2


@pytest.mark.parametrize("prec", [0, 1])
def test_residual_entry_backward_euler(lib, prec):
    """The float64 all-at-once residual ||G - A(U)||_F / ||G||_F of the
    library (Section 1's equation with M; the residual test of Algorithm 3)
    equals the oracle's, for the exact solution and for a perturbed U, in 1D
    (FEM, with a mass matrix) and 2D (5-point FD)."""
    from oracle.spatial import problem_matrices as pm
    cases = [wl.heat_1d("fem1", 255, 64, 1.0, 1.0, np.random.default_rng(2), True),
             wl.heat_2d(31, 16, 0.1, 1.0, np.random.default_rng(3))]
    for p in cases:
        Msp, Ksp = pm(p)
        Uex = modal.modal_solution(p)
        Upert = Uex + 1e-3 * np.random.default_rng(4).standard_normal(Uex.shape)
        plan = plan_for(lib, p, precision=prec, dims=p.dims)
        try:
            for Uin in (Uex, Upert):
                got = lib.paradiag_residual(plan, T(p.u0), T(p.F), T(Uin))
                _, ref = allatonce.residual(Msp, Ksp, p.tau, p.u0, p.F, Uin)
                print("dims=%d prec=%d residual gpu=%.6e oracle=%.6e" % (p.dims, prec, got, ref))
                if Uin is Uex:
                    # the exact solution rounded to float64 leaves a residual
                    # at the rounding level of ||A|| ||U|| / ||G|| (about
                    # 1e-12 for this FEM problem), which the two sides
                    # evaluate in different orders
                    assert got < 1e-11 and ref < 1e-11
                else:
                    assert abs(got - ref) <= 1e-12 * ref
        finally:
            lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("kind,n,ell,prec", [
    ("fem1", 8192, 4096, 0),     # the float64 limits on n and ell together
    ("fd1", 16384, 256, 1),      # mixed precision at its limit on n
])
def test_maximum_sizes_sampled(lib, kind, n, ell, prec):
    """Plans at the largest sizes the library accepts solve to 1e-8 against
    the exact modal solution, on sampled outputs (the full U is 2^25 values)."""
    p = make_problem(kind, n, ell, 17)
    U, info = _solve(lib, p, prec=prec, tol=1e-8)
    rng = np.random.default_rng(1)
    tt = rng.integers(0, p.ell, 3000)
    ii = rng.integers(0, p.n, 3000)
    tt[:4] = [0, 0, p.ell - 1, p.ell - 1]      # the first and last rows and points
    ii[:4] = [0, p.n - 1, 0, p.n - 1]
    ref = modal.modal_sample(p, tt, ii)
    err = np.linalg.norm(U[tt, ii] - ref) / np.linalg.norm(ref)
    print("%s n=%d ell=%d prec=%d err=%.3e res=%.3e gmres=%d sweeps=%d" % (
        kind, n, ell, prec, err, info.rel_residual, info.gmres_iters, info.sweeps))
    assert err < 1e-8, (err, info.as_dict())
    assert 0.0 <= info.rel_residual < 1e-8


@pytest.mark.parametrize("n,ell", [(300, 64), (1500, 128), (5000, 256)])
def test_autotuned_plan(lib, n, ell):
    """An autotuned plan picks a valid tile width and rows per thread, solves
    to the same accuracy as the built-in choice, and a second plan of the
    same shape reuses the choice."""
    p = make_problem("fem1", n, ell, 11)
    s = torch.cuda.current_stream().cuda_stream
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, stream=s, autotune=1)
    plan2 = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, stream=s, autotune=1)
    try:
        C, MR = lib.paradiag_plan_config(plan)
        assert C in (1, 2, 4, 8, 16, 32) and MR in (4, 8, 16)
        assert lib.paradiag_plan_config(plan2) == (C, MR)
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, 1e-10)
        torch.cuda.synchronize()
        assert allatonce.rel_err(U.cpu().numpy(), modal.modal_solution(p)) < 1e-9
        assert info.gmres_iters >= 1
    finally:
        lib.paradiag_plan_destroy(plan)
        lib.paradiag_plan_destroy(plan2)


def _mnorm_rel_err(p, U, Uex):
    """||M^1/2 (Uex - U)||_F / ||M^1/2 U||_F (x^T M x summed over time rows)."""
    Msp, _ = problem_matrices(p)
    E = Uex - U
    num = float(np.sum(E * np.asarray((Msp @ E.T).T)))
    den = float(np.sum(U * np.asarray((Msp @ U.T).T)))
    return np.sqrt(num / den)


@pytest.mark.parametrize("case,prec", [("fd1", 0), ("fem1", 0), ("fem1-ill", 0), ("fd2", 0),
                                       ("fem1", 1), ("fd2", 1)])
def test_error_bound_holds(lib, case, prec):
    """info.est_rel_error bounds the M-norm error against the exact discrete
    solution (oracle's modal form): each backward-Euler step is an M-norm
    contraction for SPD M and SPSD K, so sqrt(ell (ell+1) / 2)
    sqrt(kappa(M)) ||R|| / ||M U|| bounds it (kappa by Gershgorin)."""
    rng = np.random.default_rng(31)
    dims = 1
    if case == "fd1":
        p = wl.heat_1d("fd1", 63, 32, 1.0, 1.0, rng, True)
    elif case == "fem1":
        p = wl.heat_1d("fem1", 255, 64, 1.0, 1.0, rng, True)
    elif case == "fem1-ill":
        p = wl.heat_1d("fem1", 1023, 256, 1.0, 1e-3, rng, True)
    else:
        p, dims = wl.heat_2d(31, 16, 0.1, 1.0, rng), 2
    U, info = _solve(lib, p, prec=prec, tol=1e-10, dims=dims)
    err = _mnorm_rel_err(p, U, modal.modal_solution(p))
    assert info.rel_residual >= 0 and info.est_rel_error > 0, info.as_dict()
    assert err <= info.est_rel_error, (err, info.as_dict())
    assert info.est_rel_error < 1e-5, info.as_dict()      # and it is informative


def test_error_bound_absent_when_not_applicable(lib):
    """A non-symmetric K (a convection term) or a BDF plan: no bound (-1)."""
    import dataclasses
    p = wl.heat_1d("fd1", 63, 32, 1.0, 1.0, np.random.default_rng(32), True)
    U, info = _solve(lib, p, tol=1e-10)
    assert info.est_rel_error > 0
    lower, diag, upper = (np.array(a, dtype=np.float64) for a in p.K)
    q = dataclasses.replace(p, K=(lower, diag, 0.9 * upper))     # K no longer symmetric
    U, info = _solve(lib, q, tol=1e-10)
    assert info.rel_residual >= 0 and info.est_rel_error == -1.0, info.as_dict()
    b = dataclasses.replace(p, u0=np.tile(p.u0, (2, 1)))         # BDF2: s = 2 starting values
    U, info = _solve(lib, b, tol=1e-10, bdf_order=2)
    assert info.est_rel_error == -1.0, info.as_dict()
