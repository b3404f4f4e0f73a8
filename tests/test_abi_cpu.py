"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function that include/paradiag.h declares, and argument
validation rejects bad input before any device work."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paradiag.h")
LIB = os.path.join(ROOT, "paper_2304_12597_amd", "libparadiag.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:paradiag|pd_server|pd_admission)_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_2304_12597_amd import build
        build.build()
    return LIB


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("paradiag_plan_create", "paradiag_solve", "paradiag_solve_batch",
                 "paradiag_plan_destroy", "paradiag_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_library_marks_its_stages_for_profilers(built):
    """The solve's host stages are roctx ranges (rocprofv3 --marker-trace):
    the library imports the push/pop pair and names its ranges."""
    out = subprocess.run(["nm", "-D", "--undefined-only", built], capture_output=True,
                         text=True, check=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
    blob = open(built, "rb").read()
    for name in (b"paradiag_solve", b"paradiag: pass B (shifted solves, b)",
                 b"paradiag: capacitance GMRES (enqueued ahead)", b"paradiag: refinement sweep"):
        assert name in blob, name


def test_binding_has_every_declared_name(built):
    from paper_2304_12597_amd import binding
    for f in declared_functions():
        assert hasattr(binding, f), f


def _fd(n):
    from paper_2304_12597_amd import workloads as wl
    return wl.fd_laplacian(n, 1.0)


@pytest.mark.parametrize("kw,status", [
    (dict(ell=24), "PD_ENOTSUP"),        # not a power of two
    (dict(ell=1), "PD_EINVAL"),
    (dict(ell=8192), "PD_EINVAL"),
    (dict(tau=0.0), "PD_EINVAL"),
    (dict(tau=float("nan")), "PD_EINVAL"),
    (dict(alpha=0.0), "PD_EINVAL"),
    (dict(alpha=1.5), "PD_EINVAL"),
    (dict(maxit=0), "PD_EINVAL"),
    (dict(dims=3), "PD_EINVAL"),
    (dict(n=1), "PD_EINVAL"),
    (dict(n=9000), "PD_ENOTSUP"),        # FP64 1D limit
    (dict(precision=7), "PD_EINVAL"),
])
def test_plan_create_rejects_bad_arguments(built, kw, status):
    from paper_2304_12597_amd import binding as pd
    args = dict(n=15, ell=8, tau=0.1)
    args.update({k: kw[k] for k in ("n", "ell", "tau") if k in kw})
    opts = {k: v for k, v in kw.items() if k not in ("n", "ell", "tau")}
    with pytest.raises(pd.PDError) as ei:
        pd.paradiag_plan_create(args["n"], args["ell"], args["tau"], None, _fd(args["n"]),
                                **opts)
    assert pd.STATUS_NAMES[ei.value.status] == status
    assert pd.paradiag_last_error() != ""


def test_plan_create_rejects_nonfinite_matrix(built):
    from paper_2304_12597_amd import binding as pd
    K = [a.copy() for a in _fd(15)]
    K[1][3] = np.inf
    with pytest.raises(pd.PDError) as ei:
        pd.paradiag_plan_create(15, 8, 0.1, None, K)
    assert ei.value.status == pd.PD_EINVAL
