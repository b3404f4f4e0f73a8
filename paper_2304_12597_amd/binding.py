"""Thin ctypes binding of libparadiag (include/paradiag.h), same names.

Only argument marshalling happens here: torch tensors are passed by their
device pointers, every stage runs in the HIP library.  Importing this module
fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparadiag.so")

PD_OK, PD_EINVAL, PD_ENOMEM, PD_EHIP, PD_ENOTCONV, PD_ESINGULAR, \
    PD_ENONFINITE, PD_EBUDGET, PD_ENOTSUP = range(9)
STATUS_NAMES = ["PD_OK", "PD_EINVAL", "PD_ENOMEM", "PD_EHIP", "PD_ENOTCONV",
                "PD_ESINGULAR", "PD_ENONFINITE", "PD_EBUDGET", "PD_ENOTSUP"]
PD_FP64, PD_MIXED, PD_FP32 = 0, 1, 2
PD_SHIFTED_PARTITION, PD_SHIFTED_SINE = 0, 1
PD_KRYLOV_GMRES, PD_KRYLOV_FOM = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError("libparadiag.so is not built (run __graft_entry__.build())")
# torch brings its own HIP and HSA runtime libraries (same sonames as the
# ones the library links); load them first, so that the library binds to
# that one runtime instead of starting a second one in the process
import torch  # noqa: E402,F401
_lib = ctypes.CDLL(LIB_PATH)

_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class pd_tridiag(ctypes.Structure):
    _fields_ = [("lower", _dp), ("diag", _dp), ("upper", _dp)]


class pd_options(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int), ("precision", ctypes.c_int),
                ("alpha", ctypes.c_double), ("maxit", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("check_residual", ctypes.c_int),
                ("stream", _vp), ("autotune", ctypes.c_int),
                ("early_exit", ctypes.c_int), ("shifted_solver", ctypes.c_int),
                ("krylov", ctypes.c_int), ("fom_q", ctypes.c_int),
                ("bdf_order", ctypes.c_int)]


class pd_info(ctypes.Structure):
    _fields_ = [("gmres_iters", ctypes.c_int), ("sweeps", ctypes.c_int),
                ("pint_loops", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("gmres_rel_residual", ctypes.c_double), ("early_exit", ctypes.c_int),
                ("est_rel_error", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _sig(name, restype, argtypes):
    fn = getattr(_lib, name)
    fn.restype = restype
    fn.argtypes = argtypes
    return fn


_default_options = _sig("paradiag_default_options", None, [ctypes.POINTER(pd_options)])
_plan_create = _sig("paradiag_plan_create", ctypes.c_int,
                    [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_double,
                     ctypes.POINTER(pd_tridiag), ctypes.POINTER(pd_tridiag),
                     ctypes.POINTER(pd_options)])
_solve = _sig("paradiag_solve", ctypes.c_int,
              [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.POINTER(pd_info)])
_solve_batch = _sig("paradiag_solve_batch", ctypes.c_int,
                    [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                     ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_double,
                     ctypes.POINTER(pd_info)])
_plan_destroy = _sig("paradiag_plan_destroy", ctypes.c_int, [_vp])
_plan_config = _sig("paradiag_plan_config", ctypes.c_int,
                    [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)])
_last_error = _sig("paradiag_last_error", ctypes.c_char_p, [])
_spectrum_bytes = _sig("paradiag_spectrum_bytes", ctypes.c_size_t, [_vp])
_forward = _sig("paradiag_forward_transform", ctypes.c_int, [_vp, _vp, _vp, _vp])
_sine = _sig("paradiag_sine_transform", ctypes.c_int, [_vp, _vp, _vp])
_shifted = _sig("paradiag_shifted_solve", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp])
_cap_apply = _sig("paradiag_capacitance_apply", ctypes.c_int, [_vp, _vp, _vp])
_cap_solve = _sig("paradiag_capacitance_solve", ctypes.c_int,
                  [_vp, _vp, _vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int),
                   ctypes.POINTER(ctypes.c_double)])
_inverse = _sig("paradiag_inverse_transform", ctypes.c_int, [_vp, _vp, _vp])
_residual = _sig("paradiag_residual", ctypes.c_int,
                 [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)])


_residual_noalloc = _sig("paradiag_residual_noalloc", ctypes.c_int,
                         [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)])


class PDError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _last_error().decode(errors="replace")
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES[status] if 0 <= status < 9
                                         else status, msg))


def _check(status, where, allow=()):
    if status != PD_OK and status not in allow:
        raise PDError(status, where)
    return status


def _ptr(x):
    """Device pointer of a tensor (or an int / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return x.data_ptr()


def _tridiag(t, keep):
    if t is None:
        return None
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in t]
    keep.extend(arrs)
    s = pd_tridiag(*(a.ctypes.data_as(_dp) for a in arrs))
    keep.append(s)
    return ctypes.pointer(s)


def paradiag_default_options() -> pd_options:
    o = pd_options()
    _default_options(ctypes.byref(o))
    return o


def paradiag_last_error() -> str:
    return _last_error().decode(errors="replace")


def paradiag_plan_create(n, ell, tau, M, K, options=None, **kw):
    """M, K: (lower, diag, upper) arrays or None for M = I.  Keyword
    arguments override fields of pd_options (dims, precision, alpha, maxit,
    max_sweeps, check_residual, stream, autotune, early_exit, shifted_solver, krylov,
    fom_q, bdf_order)."""
    opt = options if options is not None else paradiag_default_options()
    for k, v in kw.items():
        if k == "stream" and v is not None and not isinstance(v, int):
            v = v.cuda_stream
        setattr(opt, k, v)
    keep = []
    plan = _vp()
    st = _plan_create(ctypes.byref(plan), int(n), int(ell), float(tau), _tridiag(M, keep),
                      _tridiag(K, keep), ctypes.byref(opt))
    _check(st, "paradiag_plan_create")
    return plan


_plan_check = _sig("paradiag_plan_check", ctypes.c_int,
                   [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(pd_tridiag),
                    ctypes.POINTER(pd_tridiag), ctypes.POINTER(pd_options)])


def paradiag_plan_check(n, ell, tau, M, K, options=None, **kw):
    """Host-only validation of a plan's problem and options; returns the
    pd_status code (no exception) and touches no GPU."""
    opt = options if options is not None else paradiag_default_options()
    for k, v in kw.items():
        setattr(opt, k, v)
    keep = []
    return int(_plan_check(int(n), int(ell), float(tau), _tridiag(M, keep), _tridiag(K, keep),
                           ctypes.byref(opt)))


def paradiag_plan_config(plan):
    """(point pairs per time-transform tile, rows per thread of the shifted
    solves) of a plan."""
    c, mr = ctypes.c_int(), ctypes.c_int()
    _check(_plan_config(plan, ctypes.byref(c), ctypes.byref(mr)), "paradiag_plan_config")
    return c.value, mr.value


def paradiag_plan_destroy(plan):
    return _check(_plan_destroy(plan), "paradiag_plan_destroy")


def paradiag_solve(plan, u0, F, U, tol, allow_notconv=False):
    info = pd_info()
    st = _solve(plan, _ptr(u0), _ptr(F), _ptr(U), float(tol), ctypes.byref(info))
    _check(st, "paradiag_solve", (PD_ENOTCONV,) if allow_notconv else ())
    return info


def paradiag_solve_batch(plans, u0s, Fs, Us, tol, allow_notconv=False):
    n = len(plans)
    arr = lambda xs: (_vp * n)(*[_ptr(x) for x in xs])
    infos = (pd_info * n)()
    st = _solve_batch((_vp * n)(*[p.value for p in plans]), n, arr(u0s), arr(Fs), arr(Us),
                      float(tol), infos)
    _check(st, "paradiag_solve_batch", (PD_ENOTCONV,) if allow_notconv else ())
    return list(infos)


def paradiag_spectrum_bytes(plan) -> int:
    return int(_spectrum_bytes(plan))


def paradiag_sine_transform(plan, inp, out):
    return _check(_sine(plan, _ptr(inp), _ptr(out)), "paradiag_sine_transform")


def paradiag_forward_transform(plan, u0, F, Hhat):
    return _check(_forward(plan, _ptr(u0), _ptr(F), _ptr(Hhat)), "paradiag_forward_transform")


def paradiag_shifted_solve(plan, Hhat, x, Uhat, b):
    return _check(_shifted(plan, _ptr(Hhat), _ptr(x), _ptr(Uhat), _ptr(b)),
                  "paradiag_shifted_solve")


def paradiag_capacitance_apply(plan, v, Jv):
    return _check(_cap_apply(plan, _ptr(v), _ptr(Jv)), "paradiag_capacitance_apply")


def paradiag_capacitance_solve(plan, b, x, rtol, allow_notconv=False):
    its = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = _cap_solve(plan, _ptr(b), _ptr(x), float(rtol), ctypes.byref(its), ctypes.byref(rr))
    _check(st, "paradiag_capacitance_solve", (PD_ENOTCONV,) if allow_notconv else ())
    return its.value, rr.value


def paradiag_inverse_transform(plan, Uhat, U):
    return _check(_inverse(plan, _ptr(Uhat), _ptr(U)), "paradiag_inverse_transform")


def paradiag_residual_noalloc(plan, u0, F, U) -> float:
    r = ctypes.c_double(-1.0)
    _check(_residual_noalloc(plan, _ptr(u0), _ptr(F), _ptr(U), ctypes.byref(r)),
           "paradiag_residual_noalloc")
    return r.value


def paradiag_residual(plan, u0, F, U) -> float:
    rel = ctypes.c_double(0.0)
    _check(_residual(plan, _ptr(u0), _ptr(F), _ptr(U), ctypes.byref(rel)), "paradiag_residual")
    return rel.value


# ---- serving ---------------------------------------------------------------

class pd_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("ell", ctypes.c_int), ("tau", ctypes.c_double),
                ("M", ctypes.POINTER(pd_tridiag)), ("K", ctypes.POINTER(pd_tridiag)),
                ("opt", pd_options), ("u0", _vp), ("F", _vp), ("U", _vp),
                ("tol", ctypes.c_double)]


_server_create = _sig("pd_server_create", ctypes.c_int,
                      [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_size_t])
_server_submit = _sig("pd_server_submit", ctypes.c_int,
                      [_vp, ctypes.POINTER(pd_request), ctypes.POINTER(ctypes.c_long)])
_server_wait = _sig("pd_server_wait", ctypes.c_int,
                    [_vp, ctypes.c_long, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(pd_info)])
_server_stats = _sig("pd_server_stats", ctypes.c_int,
                     [_vp, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_size_t),
                      ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long),
                      ctypes.POINTER(ctypes.c_size_t)])
_server_destroy = _sig("pd_server_destroy", ctypes.c_int, [_vp])
_plan_bytes = _sig("paradiag_plan_bytes", ctypes.c_size_t,
                   [ctypes.c_int, ctypes.c_int, ctypes.POINTER(pd_options)])


def paradiag_plan_bytes(n, ell, options=None, **kw):
    opt = options if options is not None else paradiag_default_options()
    for k, v in kw.items():
        setattr(opt, k, v)
    return int(_plan_bytes(int(n), int(ell), ctypes.byref(opt)))


def pd_server_create(workers, budget_bytes):
    s = _vp()
    _check(_server_create(ctypes.byref(s), int(workers), int(budget_bytes)), "pd_server_create")
    return s


def pd_server_submit(server, n, ell, tau, M, K, u0, F, U, tol, options=None, **kw):
    """Queue one solve; returns the ticket.  The tensors must stay alive until
    pd_server_wait reports the ticket done."""
    opt = options if options is not None else paradiag_default_options()
    for k, v in kw.items():
        setattr(opt, k, v)
    keep = []
    req = pd_request(int(n), int(ell), float(tau), _tridiag(M, keep) or
                     ctypes.POINTER(pd_tridiag)(), _tridiag(K, keep), opt, _ptr(u0), _ptr(F),
                     _ptr(U), float(tol))
    t = ctypes.c_long(-1)
    _check(_server_submit(server, ctypes.byref(req), ctypes.byref(t)), "pd_server_submit")
    return t.value


def pd_server_wait(server, ticket, timeout_ms=-1):
    """Returns (done, status, info)."""
    done = ctypes.c_int(0)
    st = ctypes.c_int(0)
    info = pd_info()
    _check(_server_wait(server, int(ticket), int(timeout_ms), ctypes.byref(done),
                        ctypes.byref(st), ctypes.byref(info)), "pd_server_wait")
    return bool(done.value), st.value, info


def pd_server_stats(server):
    c = ctypes.c_long(0); pk = ctypes.c_size_t(0); h = ctypes.c_long(0)
    m = ctypes.c_long(0); cur = ctypes.c_size_t(0)
    _check(_server_stats(server, ctypes.byref(c), ctypes.byref(pk), ctypes.byref(h),
                         ctypes.byref(m), ctypes.byref(cur)), "pd_server_stats")
    return {"completed": c.value, "peak_bytes": pk.value, "cache_hits": h.value,
            "cache_misses": m.value, "current_bytes": cur.value}


def pd_server_destroy(server):
    return _check(_server_destroy(server), "pd_server_destroy")


# ---- the admission policy, replayed on the host ------------------------------

class pd_admission_event(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("id", ctypes.c_int), ("key", ctypes.c_int),
                ("create_fails", ctypes.c_int), ("io_bytes", ctypes.c_size_t),
                ("plan_bytes", ctypes.c_size_t)]


class pd_admission_outcome(ctypes.Structure):
    _fields_ = [("admitted_after", ctypes.c_int), ("cache_hit", ctypes.c_int),
                ("evicted", ctypes.c_int), ("first_victim_key", ctypes.c_int),
                ("used_after", ctypes.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_admission_replay = _sig("pd_admission_replay", ctypes.c_int,
                         [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(pd_admission_event),
                          ctypes.c_int, ctypes.POINTER(pd_admission_outcome), ctypes.c_int,
                          ctypes.POINTER(ctypes.c_size_t)])


def pd_admission_replay(budget_bytes, workers, events, nreq):
    """events: (op, id, key, create_fails, io_bytes, plan_bytes) tuples.
    Returns (list of outcome dicts indexed by request id, peak bytes)."""
    ev = (pd_admission_event * max(1, len(events)))(
        *[pd_admission_event(*e) for e in events])
    out = (pd_admission_outcome * max(1, nreq))()
    peak = ctypes.c_size_t(0)
    _check(_admission_replay(int(budget_bytes), int(workers), ev, len(events), out, int(nreq),
                             ctypes.byref(peak)), "pd_admission_replay")
    return [out[i].as_dict() for i in range(nreq)], peak.value
