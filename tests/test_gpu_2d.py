"""GPU parity of the 2D separable path (DST-I along x + line solves along y)
against the CPU oracle."""
import numpy as np
import pytest

from oracle import allatonce, dst, modal, paradiag
from oracle.spatial import problem_matrices
from paper_2304_12597_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=dev())


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def plan2d(lib, p, **kw):
    return lib.paradiag_plan_create(p.n, p.ell, p.tau, None, p.K, dims=2,
                                    stream=torch.cuda.current_stream().cuda_stream, **kw)


def dst_x(A, n):
    """Orthonormal DST-I along x of [rows][n*n] arrays (oracle sine matrix)."""
    A = np.asarray(A)
    return dst.dst1(A.reshape(A.shape[:-1] + (n, n)), axis=-1).reshape(A.shape)


# n + 1 a power of two (one FFT of length 2(n+1) per pair of rows) and other
# n (the chirp-z form: FFTs of length L >= 2n - 1)
@pytest.mark.parametrize("n,ell", [(3, 4), (7, 8), (31, 32), (63, 16), (127, 8),
                                   (2, 4), (4, 4), (6, 8), (20, 8), (100, 4), (256, 2)])
@pytest.mark.parametrize("prec", [0, 2])
def test_2d_forward_transform(lib, n, ell, prec):
    p = wl.heat_2d(n, ell, 0.1, 1.0, np.random.default_rng(n))
    rng = np.random.default_rng(1)
    p.u0 = rng.standard_normal(n * n)
    p.F = rng.standard_normal((ell, n * n))
    plan = plan2d(lib, p, precision=prec)
    F2 = ell // 2 + 1
    cdt = np.complex128 if prec == 0 else np.complex64
    try:
        nb = lib.paradiag_spectrum_bytes(plan)
        H = torch.empty(nb // 8, dtype=torch.float64, device=dev())
        lib.paradiag_forward_transform(plan, T(p.u0), T(p.F), H)
        torch.cuda.synchronize()
        got = H.cpu().numpy().view(cdt).reshape(F2, n * n)
    finally:
        lib.paradiag_plan_destroy(plan)
    Hrows = p.tau * p.F
    Hrows[0] += p.u0
    ref = np.fft.fft(dst_x(Hrows, n), axis=0)[:F2]
    assert rel(got, ref) < (1e-12 if prec == 0 else 2e-5)


@pytest.mark.parametrize("n,ell", [(7, 8), (31, 16)])
def test_2d_capacitance_apply(lib, n, ell):
    p = wl.heat_2d(n, ell, 0.1, 0.05, np.random.default_rng(3))
    Msp, Ksp = problem_matrices(p)
    cap = paradiag.Capacitance(Msp, Ksp, p.tau, ell)
    v = np.random.default_rng(4).standard_normal(n * n)
    ref = dst_x(cap.matvec(dst_x(v, n)).real, n)
    plan = plan2d(lib, p)
    try:
        Jv = torch.empty(n * n, dtype=torch.float64, device=dev())
        lib.paradiag_capacitance_apply(plan, T(v), Jv)
        torch.cuda.synchronize()
        got = Jv.cpu().numpy()
    finally:
        lib.paradiag_plan_destroy(plan)
    assert rel(got, ref) < 1e-12


def _solve(lib, p, prec=0, tol=1e-10, **kw):
    plan = plan2d(lib, p, precision=prec, check_residual=1, **kw)
    try:
        U = torch.empty((p.ell, p.nbar), dtype=torch.float64, device=dev())
        info = lib.paradiag_solve(plan, T(p.u0), T(p.F), U, tol)
        torch.cuda.synchronize()
        return U.cpu().numpy(), info
    finally:
        lib.paradiag_plan_destroy(plan)


@pytest.mark.parametrize("n,ell,nu,T_,bound", [(3, 2, 1.0, 0.1, 1e-10), (7, 8, 1.0, 0.1, 1e-10),
                                               (31, 64, 0.01, 1.0, 1e-10),
                                               (127, 16, 1.0, 0.1, 1e-10),
                                               (63, 256, 0.001, 0.1, 1e-9),
                                               (2, 4, 1.0, 0.1, 1e-10), (6, 8, 1.0, 0.1, 1e-10),
                                               (20, 16, 0.1, 1.0, 1e-10),
                                               (100, 16, 1.0, 0.1, 1e-10)])
def test_2d_end_to_end_fp64(lib, n, ell, nu, T_, bound):
    """nu*T = 1e-4 makes J_ell ill-conditioned (Theorem 1 bound
    1 + 1/(tau lambda_min) ~ 1e5): the solve uses a tighter tolerance and the
    error bound is 1e-9 there."""
    p = wl.heat_2d(n, ell, T_, nu, np.random.default_rng(n + ell))
    U, info = _solve(lib, p, tol=1e-10 if bound == 1e-10 else 1e-13)
    err = allatonce.rel_err(U, modal.modal_solution(p))
    print("2D n=%d ell=%d err=%.3e res=%.3e gmres=%d" % (n, ell, err, info.rel_residual,
                                                         info.gmres_iters))
    assert err < bound
    assert 0 <= info.rel_residual < 1e-11


def test_2d_with_source_matches_stepping(lib):
    n, ell = 15, 16
    p = wl.heat_2d(n, ell, 0.5, 0.3, np.random.default_rng(8))
    p.F = np.random.default_rng(9).standard_normal((ell, n * n))
    U, info = _solve(lib, p)
    assert allatonce.rel_err(U, allatonce.step(p)) < 1e-11


# n = 100: the refinement's fused residual and accumulating inverse run on
# the chirp-z DST along x
@pytest.mark.parametrize("n", [63, 100])
def test_2d_mixed(lib, n):
    p = wl.heat_2d(n, 32, 0.1, 1.0, np.random.default_rng(2))
    U, info = _solve(lib, p, prec=1, tol=1e-10)
    err = allatonce.rel_err(U, modal.modal_solution(p))
    assert err < 1e-8, (err, info.as_dict())


@pytest.mark.parametrize("prec", [0, 1])
def test_2d_full_size_sampled(lib, prec):
    """511 x 511 grid, ell = 256, T = 0.1 (66.9M space-time unknowns):
    sampled outputs vs the exact modal solution, float64 (1e-10) and the
    mixed form (complex64 DST/transforms/line solves, float64 refinement:
    1e-8, PD_OK, residual at most tol)."""
    p = wl.cfg_fd_2d()
    tol = 1e-10 if prec == 0 else 1e-8
    U, info = _solve(lib, p, prec=prec, tol=tol)
    rng = np.random.default_rng(0)
    tt = rng.integers(0, p.ell, 3000)
    ii = rng.integers(0, p.nbar, 3000)
    tt[:2] = [0, p.ell - 1]
    ii[:2] = [0, p.nbar - 1]
    ref = modal.modal_sample(p, tt, ii)
    err = np.linalg.norm(U[tt, ii] - ref) / np.linalg.norm(ref)
    print("2D 511^2 ell=256 prec=%d err=%.3e res=%.3e gmres=%d sweeps=%d" % (
        prec, err, info.rel_residual, info.gmres_iters, info.sweeps))
    if prec == 0:
        assert err < 1e-10, (err, info.as_dict())
        assert 0 <= info.rel_residual < 1e-11
    else:
        assert err < 1e-8, (err, info.as_dict())
        assert 0 <= info.rel_residual <= tol


# Algorithm 2 runs at T = 1: at T = 0.1 its polynomial Krylov space of the
# stiff K needs more than the 32-step cap (as for the stiff 1D workload)
@pytest.mark.parametrize("prec,krylov,T_", [(0, 0, 0.1), (1, 0, 0.1), (0, 1, 1.0)])
def test_2d_maximum_size_sampled(lib, prec, krylov, T_):
    """The largest 2D grid the library accepts (1023 x 1023, ~1.05M unknowns per
    step), ell = 32: float64 and mixed precision with GMRES, and Algorithm 2,
    on sampled outputs of the exact modal solution."""
    p = wl.heat_2d(1023, 32, T_, 1.0, np.random.default_rng(5))
    kw = {"krylov": lib.PD_KRYLOV_FOM} if krylov else {}
    U, info = _solve(lib, p, prec=prec, tol=1e-8, **kw)
    rng = np.random.default_rng(2)
    tt = rng.integers(0, p.ell, 3000)
    ii = rng.integers(0, p.nbar, 3000)
    tt[:2] = [0, p.ell - 1]
    ii[:2] = [0, p.nbar - 1]
    ref = modal.modal_sample(p, tt, ii)
    err = np.linalg.norm(U[tt, ii] - ref) / np.linalg.norm(ref)
    print("n=1023 ell=32 T=%g prec=%d krylov=%d err=%.3e res=%.3e its=%d sweeps=%d" % (
        T_, prec, krylov, err, info.rel_residual, info.gmres_iters, info.sweeps))
    assert err < 1e-8, (err, info.as_dict())
    assert 0.0 <= info.rel_residual < 1e-8
