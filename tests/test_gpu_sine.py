"""GPU parity of the sine-basis shifted solves (PD_SHIFTED_SINE): the DST-I
stage against the oracle's sine matrix, and whole solves against the exact
modal solution and the oracle's stepping."""
import numpy as np
import pytest

from oracle import allatonce, dst, modal
from oracle.spatial import problem_matrices
from paper_2304_12597_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=dev())


def sine_plan(lib, p, **kw):
    return lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K,
                                    shifted_solver=lib.PD_SHIFTED_SINE,
                                    stream=torch.cuda.current_stream().cuda_stream, **kw)


def make_problem(kind, n, ell, seed, nu=1.0, T_=1.0):
    return wl.heat_1d(kind, n, ell, T_, nu, np.random.default_rng(seed), True)


# n + 1 a power of two, and other n (chirp-z form, n <= 4095)
@pytest.mark.parametrize("n,ell", [(15, 2), (31, 4), (63, 8), (255, 64), (1023, 16),
                                   (4095, 4), (8191, 2), (2, 2), (20, 4), (100, 4), (1000, 8),
                                   (4000, 2), (4094, 2)])
def test_sine_transform(lib, n, ell):
    p = make_problem("fd1", n, ell, n)
    plan = sine_plan(lib, p)
    try:
        x = np.random.default_rng(n + ell).standard_normal((ell, n))
        X = T(x)
        out = torch.empty_like(X)
        lib.paradiag_sine_transform(plan, X, out)
        lib.paradiag_sine_transform(plan, X, X)      # in place
        torch.cuda.synchronize()
        got, got_in_place = out.cpu().numpy(), X.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    ref = dst.dst1(x, axis=1)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-13, err
    assert np.array_equal(got, got_in_place)


def _solve(lib, p, tol=1e-10, **kw):
    plan = sine_plan(lib, p, check_residual=1, **kw)
    try:
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, tol)
        torch.cuda.synchronize()
        return U.cpu().numpy(), info
    finally:
        lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("kind,n,ell,nu", [
    ("fd1", 15, 2, 1.0), ("fd1", 31, 8, 1.0), ("fem1", 63, 32, 0.1), ("fd1", 255, 256, 1e-3),
    ("fem1", 1023, 128, 1.0), ("fd1", 2047, 1024, 0.01), ("fem1", 4095, 64, 1e-3),
    ("fd1", 127, 4096, 1.0), ("fd1", 100, 16, 1.0), ("fem1", 1000, 64, 0.1),
    ("fd1", 3000, 32, 1e-2)])
def test_sine_solve_matches_exact(lib, kind, n, ell, nu):
    """The sine-basis solve reaches the exact all-at-once solution to float64
    rounding (no elimination floor), with no Krylov iterations."""
    p = make_problem(kind, n, ell, 3 * n + ell, nu=nu)
    U, info = _solve(lib, p)
    err = allatonce.rel_err(U, modal.modal_solution(p))
    assert err < 1e-12, (err, info.as_dict())
    assert info.gmres_iters == 0 and info.pint_loops == 1
    # the float64 residual of a stiff problem is itself rounding-limited
    # (||A|| ||U|| >> ||G||); the error above is the accuracy measure
    assert 0 <= info.rel_residual < 1e-9


@pytest.mark.parametrize("alpha", [0.5, 1e-2])
def test_sine_solve_alpha(lib, alpha):
    """Algorithm 3 in the sine basis (alpha-circulant time transform): the
    correction is exact, so U solves the original system."""
    p = make_problem("fem1", 127, 64, 9, nu=0.1)
    U, info = _solve(lib, p, alpha=alpha)
    kappa = alpha ** (-(p.ell - 1) / p.ell)
    err = allatonce.rel_err(U, modal.modal_solution(p))
    assert err < 1e-13 * max(10.0, kappa), err


def test_sine_solve_matches_stepping(lib):
    p = make_problem("fem1", 511, 128, 5, nu=0.05)
    U, _ = _solve(lib, p)
    Msp, Ksp = problem_matrices(p)
    U1 = allatonce.step_1d(p.M, p.K, p.tau, p.u0, p.F)
    assert allatonce.rel_err(U, U1) < 1e-10


def test_sine_fem_full_size_sampled(lib):
    """n = 8191, ell = 2048 FEM workload: the float64 tolerance of 1e-10
    against the exact modal solution, on sampled outputs."""
    p = wl.cfg_fem_1d()
    U, info = _solve(lib, p, tol=1e-8)
    rng = np.random.default_rng(0)
    tt = rng.integers(0, p.ell, 4000)
    ii = rng.integers(0, p.n, 4000)
    ref = modal.modal_sample(p, tt, ii)
    err = np.linalg.norm(U[tt, ii] - ref) / np.linalg.norm(ref)
    assert err < 1e-10, (err, info.as_dict())
    # a dense orthogonal transform leaves rounding of order u ||U|| in every
    # mode, and A amplifies the high modes by up to tau kappa_max ~ 4e5, so
    # the float64 residual sits near 1e-7 while the error is below 1e-10
    assert 0 <= info.rel_residual < 1e-6


def test_sine_plan_rejects_unsupported(lib):
    p = make_problem("fd1", 5000, 8, 1)         # n + 1 not a power of two and n > 4095
    with pytest.raises(RuntimeError):
        sine_plan(lib, p)
    p = make_problem("fd1", 63, 8, 1)
    K = (p.K[0], p.K[1].copy(), p.K[2])
    K[1][5] *= 1.01                              # not Toeplitz
    with pytest.raises(RuntimeError):
        lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, K,
                                 shifted_solver=lib.PD_SHIFTED_SINE)
    with pytest.raises(RuntimeError):           # float64 only
        sine_plan(lib, make_problem("fd1", 63, 8, 1), precision=lib.PD_MIXED)
