"""Host-only logic of the library, on the CPU (no GPU is touched): the plan
checks that plan creation runs before any device work, including the
singular zero-frequency block of Section 2, and the serving runtime's
admission and eviction policy replayed on scripted arrivals against a fake
budget."""
import numpy as np
import pytest

from paper_2304_12597_amd import workloads as wl


@pytest.fixture(scope="module")
def pd():
    from paper_2304_12597_amd import binding
    return binding


def neumann(n, scale):
    lower, diag, upper = wl.fd_laplacian(n, 1.0)
    diag = diag.copy()
    diag[0] = diag[-1] = 0.5 * diag[1]
    return tuple(a * scale for a in (lower, diag, upper))


@pytest.mark.parametrize("n", [2, 7, 63, 8191])
@pytest.mark.parametrize("kind", ["fd1", "fem1"])
def test_plan_check_singular_zero_frequency(pd, n, kind):
    """With alpha = 1 the zero-frequency block is P_0 = tau K (Section 2:
    the shift 1 - pi_0 vanishes), so a pure-Neumann K (rows summing to zero)
    is PD_ESINGULAR; the Dirichlet K is accepted, and so is the Neumann K
    with alpha < 1 (Section 4: no shift vanishes)."""
    h = 1.0 / (n + 1)
    M = wl.fem_mass(n) if kind == "fem1" else None
    scale = h if kind == "fem1" else 1.0
    K = neumann(n, scale)
    assert pd.paradiag_plan_check(n, 16, 1.0 / 16, M, K) == pd.PD_ESINGULAR
    assert "singular" in pd.paradiag_last_error()
    assert pd.paradiag_plan_check(n, 16, 1.0 / 16, M, K, alpha=0.5) == pd.PD_OK
    Kd = tuple(a * scale for a in wl.fd_laplacian(n, 1.0))
    assert pd.paradiag_plan_check(n, 16, 1.0 / 16, M, Kd) == pd.PD_OK


def test_plan_check_singular_2d(pd):
    """2D: K = I (x) T + T (x) I is singular when two eigenvalues of T sum
    to zero; T = tridiag(o, d, o) with d = 2 |o| cos(pi / (n + 1)) makes the
    smallest one zero."""
    n = 31
    o = -1.0
    d = 2.0 * abs(o) * np.cos(np.pi / (n + 1)) / 2.0
    T = (np.full(n, o), np.full(n, d), np.full(n, o))
    assert pd.paradiag_plan_check(n, 8, 0.1, None, T, dims=2) == pd.PD_ESINGULAR
    assert pd.paradiag_plan_check(n, 8, 0.1, None, wl.fd_laplacian(n, 1.0), dims=2) == pd.PD_OK


@pytest.mark.parametrize("kw,status", [
    (dict(ell=24), "PD_ENOTSUP"), (dict(ell=8192), "PD_EINVAL"), (dict(tau=-1.0), "PD_EINVAL"),
    (dict(n=9000), "PD_ENOTSUP"), (dict(n=9000, precision=1), "PD_OK"),
    (dict(dims=2, n=2000), "PD_ENOTSUP"), (dict(bdf_order=2, precision=1), "PD_ENOTSUP"),
    (dict(shifted_solver=1, n=5000), "PD_ENOTSUP"), (dict(krylov=3), "PD_EINVAL")])
def test_plan_check_statuses(pd, kw, status):
    args = dict(n=15, ell=8, tau=0.1)
    args.update({k: kw[k] for k in ("n", "ell", "tau") if k in kw})
    opts = {k: v for k, v in kw.items() if k not in ("n", "ell", "tau")}
    st = pd.paradiag_plan_check(args["n"], args["ell"], args["tau"], None,
                                wl.fd_laplacian(args["n"], 1.0), **opts)
    assert pd.STATUS_NAMES[st] == status


# ------------------------------------------------------------- admission --

ARRIVE, FINISH = 0, 1


def ev_arrive(rid, key, io, plan):
    return (ARRIVE, rid, key, 0, io, plan)


def ev_finish(rid, fails=0):
    return (FINISH, rid, 0, fails, 0, 0)


def test_admission_fifo_budget_and_lru(pd):
    """Budget 100, 4 workers.  r0 (key 1) and r1 (key 2) fit together
    (20 + 30 each); r2 (key 3) waits; when r0 finishes its plan stays cached
    (idle, 30 bytes) and r2 is admitted only after that idle plan is evicted.
    r3 (key 2, after r1 finished) reuses r1's cached plan: a hit that needs
    only its arrays."""
    events = [ev_arrive(0, 1, 20, 30), ev_arrive(1, 2, 20, 30), ev_arrive(2, 3, 20, 30),
              ev_finish(0), ev_finish(1), ev_arrive(3, 2, 20, 30), ev_finish(2), ev_finish(3)]
    out, peak = pd.pd_admission_replay(100, 4, events, 4)
    assert [o["admitted_after"] for o in out] == [0, 1, 3, 5]
    assert out[2]["evicted"] == 1 and out[2]["first_victim_key"] == 1
    assert out[2]["used_after"] == 100
    assert out[3]["cache_hit"] == 1 and out[3]["evicted"] == 0
    # r1 finished (event 4): 100 - 20 (r1's arrays) = 80; r3 adds its 20
    assert out[3]["used_after"] == 100
    assert peak == 100


def test_admission_evicts_least_recently_used_and_keeps_the_reused_plan(pd):
    """Three idle cached plans (keys 1, 2, 3, last used in that order); a
    request for key 1 that does not fit evicts key 2 (the oldest other
    plan), never its own idle plan, which it reuses."""
    events = [ev_arrive(0, 1, 10, 20), ev_finish(0), ev_arrive(1, 2, 10, 20), ev_finish(1),
              ev_arrive(2, 3, 10, 20), ev_finish(2), ev_arrive(3, 1, 45, 20)]
    out, peak = pd.pd_admission_replay(100, 4, events, 4)
    assert out[3]["admitted_after"] == 6
    assert out[3]["cache_hit"] == 1
    assert out[3]["evicted"] == 1 and out[3]["first_victim_key"] == 2
    assert out[3]["used_after"] == 40 + 45
    assert peak <= 100


def test_admission_rejects_oversized_and_waits_for_workers(pd):
    """A request whose arrays and plan alone exceed the budget is rejected
    at arrival (PD_EBUDGET in the server); with one worker, a fitting
    request still waits for the running one (FIFO order is kept)."""
    events = [ev_arrive(0, 1, 10, 10), ev_arrive(1, 2, 200, 10), ev_arrive(2, 3, 10, 10),
              ev_finish(0), ev_finish(2)]
    out, _ = pd.pd_admission_replay(100, 1, events, 3)
    assert out[0]["admitted_after"] == 0
    assert out[1]["admitted_after"] == -2
    assert out[2]["admitted_after"] == 3


def test_admission_failed_creation_releases_reservation(pd):
    events = [ev_arrive(0, 1, 10, 60), ev_arrive(1, 2, 10, 60), ev_finish(0, fails=1)]
    out, _ = pd.pd_admission_replay(100, 4, events, 2)
    assert out[1]["admitted_after"] == 2
    assert out[1]["evicted"] == 0 and out[1]["used_after"] == 70


def test_admission_nothing_evicted_in_vain(pd):
    """If evicting every idle plan would still not make room (a busy plan
    holds the budget), nothing is evicted and the request waits."""
    events = [ev_arrive(0, 1, 10, 20), ev_finish(0), ev_arrive(1, 2, 10, 50),
              ev_arrive(2, 3, 10, 50), ev_finish(1)]
    out, _ = pd.pd_admission_replay(100, 4, events, 3)
    assert out[1]["admitted_after"] == 2 and out[1]["evicted"] == 0
    # r1's finish leaves two idle plans (keys 1 and 2, 70 bytes accounted);
    # r2 needs 60: both are evicted, the older (key 1) first
    assert out[2]["admitted_after"] == 4
    assert out[2]["evicted"] == 2 and out[2]["first_victim_key"] == 1
    assert out[2]["used_after"] == 60


def test_admission_random_invariants(pd):
    """Random scripts: the accounted bytes never exceed the budget, every
    admitted request is admitted in arrival order, and a request never
    waits while the head of the queue is admissible."""
    rng = np.random.default_rng(0)
    for trial in range(20):
        nreq = 60
        events, running, arrived = [], [], 0
        while arrived < nreq or running:
            if arrived < nreq and (not running or rng.uniform() < 0.6):
                events.append(ev_arrive(arrived, int(rng.integers(0, 6)),
                                        int(rng.integers(1, 40)), int(rng.integers(1, 60))))
                arrived += 1
            # finish only requests the policy must have admitted: replay so far
            out, _ = pd.pd_admission_replay(128, 3, events, nreq)
            running = [i for i in range(arrived) if out[i]["admitted_after"] >= 0 and
                       not any(e[0] == FINISH and e[1] == i for e in events)]
            if running and (arrived == nreq or rng.uniform() < 0.5):
                events.append(ev_finish(int(rng.choice(running)), int(rng.uniform() < 0.1)))
            if arrived == nreq and not running:
                waiting = [i for i in range(nreq) if out[i]["admitted_after"] == -1]
                assert not waiting
        out, peak = pd.pd_admission_replay(128, 3, events, nreq)
        assert peak <= 128
        order = [o["admitted_after"] for o in out if o["admitted_after"] >= 0]
        assert order == sorted(order)
        assert all(o["used_after"] <= 128 for o in out)
