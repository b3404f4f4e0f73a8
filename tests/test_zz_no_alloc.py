"""The allocation-free residual entry point (paradiag_residual_noalloc)
against paradiag_residual, through the C ABI: two calls in a row on the
shared static scratch, the second with a smaller problem, for an exact and
a perturbed U, in 1D (FEM, the largest partial-norm count) and 2D."""
import numpy as np
import pytest

from oracle import modal
from paper_2304_12597_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.tensor(np.ascontiguousarray(a), device=dev())


def _case(lib, p, seed):
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, dims=p.dims,
                                    stream=torch.cuda.current_stream().cuda_stream)
    Uex = modal.modal_solution(p)
    Upert = Uex + 1e-4 * np.random.default_rng(seed).standard_normal(Uex.shape)
    return plan, [(T(p.u0), T(p.F), T(U)) for U in (Uex, Upert)]


def test_residual_noalloc_matches_residual(lib):
    big = wl.heat_1d("fem1", 4095, 512, 1.0, 1.0, np.random.default_rng(1), True)   # 8192 blocks
    small = wl.heat_1d("fd1", 63, 8, 1.0, 1.0, np.random.default_rng(2), True)      # 2 blocks
    flat = wl.heat_2d(31, 16, 0.1, 1.0, np.random.default_rng(3))
    for p, seed in ((big, 4), (small, 5), (flat, 6), (small, 7)):
        plan, arrays = _case(lib, p, seed)
        try:
            for u0, F, U in arrays:
                ref = lib.paradiag_residual(plan, u0, F, U)
                got = lib.paradiag_residual_noalloc(plan, u0, F, U)
                print("n=%d ell=%d dims=%d residual %.6e noalloc %.6e" % (
                    p.n, p.ell, p.dims, ref, got))
                assert np.isfinite(got) and got >= 0.0
                # the same partial norms, summed in a different fixed order
                assert abs(got - ref) <= 1e-12 * ref + 1e-300, (got, ref)
        finally:
            lib.paradiag_plan_destroy(plan)


def test_residual_noalloc_rejects_bdf_plans(lib):
    p = wl.heat_1d("fem1", 63, 16, 1.0, 1.0, np.random.default_rng(8), True)
    plan = lib.paradiag_plan_create(p.n, p.ell, p.tau, p.M, p.K, bdf_order=2,
                                    stream=torch.cuda.current_stream().cuda_stream)
    try:
        u0 = T(np.tile(p.u0, (2, 1)))
        U = torch.zeros((p.ell, p.nbar), dtype=torch.float64, device=dev())
        with pytest.raises(lib.PDError) as ei:
            lib.paradiag_residual_noalloc(plan, u0, T(p.F), U)
        assert ei.value.status == lib.PD_ENOTSUP
    finally:
        lib.paradiag_plan_destroy(plan)
