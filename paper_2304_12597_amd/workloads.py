"""Seeded synthetic heat problems: the inputs both the GPU path and the oracle read.

This module only *builds inputs*: grids, the spatial matrices M and K that
define the problem (the user-side discretisation that the method takes as
input, Section 1, all-at-once backward Euler equation), the nodal initial
value u0 and the nodal source values f(t_j).  It contains none of the
method's arithmetic (no transforms, no shifted solves, no time stepping, no
eigenvalues).

Conventions
-----------
* Space-time arrays are time-major: ``F[j, i]`` is f at time t_{j+1} =
  (j+1)*tau at spatial node i (so row j is the (j+1)-st column of the
  paper's n-bar x ell matrix).  The paper evaluates f at the backward-Euler
  times t_j = j*tau, j = 1..ell.
* Tridiagonal matrices are three length-n arrays ``(lower, diag, upper)``;
  ``lower[i]`` multiplies x[i-1] in row i and ``upper[i]`` multiplies
  x[i+1]; ``lower[0]`` and ``upper[n-1]`` are zero.
* 2D grids are n x n interior points of (0,1)^2 with h = 1/(n+1), flattened
  row-major: node (y, x) has index y*n + x.  K = I (x) T + T (x) I with the
  1D operator T given as a tridiagonal; M = I.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64).  Per problem the
draw order is: n, ell, nu (ensembles only), then the initial-value
coefficients (k = 2..8 in 1D; (k, m) row-major in 2D), then the source
amplitudes a_k (k = 1..16), then the source frequencies b_k (k = 1..16).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np

Tridiag = Tuple[np.ndarray, np.ndarray, np.ndarray]


@dataclass
class HeatProblem:
    """One all-at-once backward-Euler heat problem (1D or 2D)."""

    kind: str                  # "fd1", "fem1" or "fd2"
    n: int                     # interior points (per side in 2D)
    ell: int                   # number of time steps
    T: float                   # final time
    nu: float                  # diffusion coefficient
    M: Optional[Tridiag]       # 1D mass matrix (None = identity)
    K: Tridiag                 # 1D stiffness matrix (2D: the 1D factor T)
    u0: np.ndarray             # [nbar] nodal initial value
    F: np.ndarray              # [ell, nbar] nodal source at t_1..t_ell
    # sine-series description of the data (used by the modal oracle)
    u0_modes: dict = field(default_factory=dict)   # k or (k, m) -> coefficient
    src_a: np.ndarray = field(default_factory=lambda: np.zeros(0))
    src_b: np.ndarray = field(default_factory=lambda: np.zeros(0))
    seed: int = 0

    @property
    def dims(self) -> int:
        return 2 if self.kind == "fd2" else 1

    @property
    def nbar(self) -> int:
        return self.n * self.n if self.dims == 2 else self.n

    @property
    def tau(self) -> float:
        return self.T / self.ell

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def unknowns(self) -> int:
        return self.nbar * self.ell


# --------------------------------------------------------------------------
# spatial matrices (problem definition)
# --------------------------------------------------------------------------

def _const_tridiag(n: int, off: float, mid: float) -> Tridiag:
    lower = np.full(n, off, dtype=np.float64)
    upper = np.full(n, off, dtype=np.float64)
    lower[0] = 0.0
    upper[-1] = 0.0
    return lower, np.full(n, mid, dtype=np.float64), upper


def fd_laplacian(n: int, nu: float) -> Tridiag:
    """nu * tridiag(-1, 2, -1) / h^2, second-order finite differences."""
    h = 1.0 / (n + 1)
    return _const_tridiag(n, -nu / h**2, 2.0 * nu / h**2)


def fem_stiffness(n: int, nu: float) -> Tridiag:
    """nu * tridiag(-1, 2, -1) / h, P1 finite elements."""
    h = 1.0 / (n + 1)
    return _const_tridiag(n, -nu / h, 2.0 * nu / h)


def fem_mass(n: int) -> Tridiag:
    """(h/6) tridiag(1, 4, 1), consistent P1 mass matrix."""
    h = 1.0 / (n + 1)
    return _const_tridiag(n, h / 6.0, 4.0 * h / 6.0)


# --------------------------------------------------------------------------
# nodal data
# --------------------------------------------------------------------------

def grid_1d(n: int) -> np.ndarray:
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def _u0_1d(x: np.ndarray, c: np.ndarray) -> Tuple[np.ndarray, dict]:
    """u0 = sin(pi x) + sum_{k=2..8} c_k sin(k pi x) / k^2."""
    u0 = np.sin(np.pi * x)
    modes = {1: 1.0}
    for idx, k in enumerate(range(2, 9)):
        coef = c[idx] / k**2
        u0 = u0 + coef * np.sin(k * np.pi * x)
        modes[k] = float(coef)
    return u0, modes


def _source_1d(x: np.ndarray, ell: int, tau: float, a: np.ndarray,
               b: np.ndarray) -> np.ndarray:
    """f(x, t_j) = sum_{k=1..16} a_k sin(k pi x) cos(b_k t_j), j = 1..ell."""
    t = tau * np.arange(1, ell + 1, dtype=np.float64)
    k = np.arange(1, a.size + 1, dtype=np.float64)
    amp = a[None, :] * np.cos(np.outer(t, b))        # [ell, K]
    modes = np.sin(np.outer(k, np.pi * x))            # [K, n]
    return amp @ modes


def heat_1d(kind: str, n: int, ell: int, T: float, nu: float,
            rng: np.random.Generator, with_source: bool) -> HeatProblem:
    """1D heat problem on (0,1), zero Dirichlet data, seeded sine-series data."""
    assert kind in ("fd1", "fem1")
    x = grid_1d(n)
    c = rng.standard_normal(7)
    if with_source:
        a = rng.standard_normal(16)
        b = rng.uniform(0.0, 10.0, 16)
    else:
        a = np.zeros(0)
        b = np.zeros(0)
    u0, modes = _u0_1d(x, c)
    tau = T / ell
    F = _source_1d(x, ell, tau, a, b) if with_source else np.zeros((ell, n))
    if kind == "fd1":
        M, K = None, fd_laplacian(n, nu)
    else:
        M, K = fem_mass(n), fem_stiffness(n, nu)
    return HeatProblem(kind, n, ell, T, nu, M, K, u0, F, modes, a, b)


def heat_2d(n: int, ell: int, T: float, nu: float,
            rng: np.random.Generator) -> HeatProblem:
    """2D heat on (0,1)^2, 5-point FD, f = 0,
    u0 = sum_{k,m<=8} c_km sin(k pi x) sin(m pi y) / (k^2 + m^2)."""
    x = grid_1d(n)
    c = rng.standard_normal((8, 8))
    u0 = np.zeros((n, n))            # [y, x]
    modes = {}
    for k in range(1, 9):            # x-mode
        sx = np.sin(k * np.pi * x)
        for m in range(1, 9):        # y-mode
            sy = np.sin(m * np.pi * x)
            coef = c[k - 1, m - 1] / (k * k + m * m)
            u0 += coef * np.outer(sy, sx)
            modes[(k, m)] = float(coef)
    return HeatProblem("fd2", n, ell, T, nu, None, fd_laplacian(n, nu),
                       u0.reshape(-1), np.zeros((ell, n * n)), modes,
                       np.zeros(0), np.zeros(0))


# --------------------------------------------------------------------------
# the five workload families
# --------------------------------------------------------------------------

def cfg_small_fd(seed: int = 0, n: int = 63, ell: int = 32) -> HeatProblem:
    """1D FD heat, n = 63 (h = 1/64), ell = 32, T = 1, nu = 1, f = 0."""
    p = heat_1d("fd1", n, ell, 1.0, 1.0, np.random.default_rng(seed), False)
    p.seed = seed
    return p


def cfg_fem_1d(seed: int = 1, n: int = 8191, ell: int = 2048) -> HeatProblem:
    """1D P1-FEM heat, n = 8191, ell = 2048, T = 1, nu = 1, 16-mode source."""
    p = heat_1d("fem1", n, ell, 1.0, 1.0, np.random.default_rng(seed), True)
    p.seed = seed
    return p


def cfg_fd_2d(seed: int = 2, n: int = 511, ell: int = 256) -> HeatProblem:
    """2D 5-point FD heat, 511 x 511 interior grid, ell = 256, T = 0.1, f = 0."""
    p = heat_2d(n, ell, 0.1, 1.0, np.random.default_rng(seed))
    p.seed = seed
    return p


ENSEMBLE_ELLS = (64, 128, 256, 512, 1024)


def ensemble_params(seed: int = 3, count: int = 512):
    """(n, ell, nu) triples of the 1D FD ensemble; the rest of each problem's
    draws follow in the same generator (see ``ensemble``)."""
    return [(p.n, p.ell, p.nu) for p in ensemble(seed, count, build=False)]


def ensemble(seed: int = 3, count: int = 512, build: bool = True,
             n_range=(255, 4095)):
    """Ensemble of independent 1D FD heat problems: n ~ U{255..4095},
    ell uniform in {64,...,1024}, nu log-uniform in [1e-3, 1], T = 1,
    u0 and f as in the FEM workload."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        ell = int(ENSEMBLE_ELLS[int(rng.integers(0, len(ENSEMBLE_ELLS)))])
        nu = float(np.exp(rng.uniform(np.log(1e-3), np.log(1.0))))
        if build:
            p = heat_1d("fd1", n, ell, 1.0, nu, rng, True)
        else:
            rng.standard_normal(7); rng.standard_normal(16); rng.uniform(0, 10, 16)
            p = HeatProblem("fd1", n, ell, 1.0, nu, None, (np.zeros(0),) * 3,
                            np.zeros(0), np.zeros((0, 0)))
        p.seed = seed
        out.append(p)
    return out


@dataclass
class Request:
    arrival: float            # seconds after stream start
    problem: HeatProblem


def iter_serving_stream(seed: int = 4, count: int = 64, rate: float = 100.0,
                        fem_n=(1023, 16383), fem_ells=(128, 256, 512, 1024, 2048),
                        sides=(127, 255, 511), fd2_ells=(64, 128, 256, 512), build=True):
    """Poisson arrivals at ``rate`` requests/s of mixed requests: 70% 1D FEM
    heat (n ~ U{1023..16383}, ell a power of two in 128..2048, T = 1, with
    source) and 30% 2D FD heat (side in {127, 255, 511}, ell in 64..512,
    T = 0.1, f = 0), nu log-uniform in [1e-3, 1].  Yields one Request at a
    time.  build=False draws the same stream but leaves the problems' arrays
    empty (sizes only); a set of request indices builds only those."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for idx in range(count):
        make = build if isinstance(build, bool) else idx in build
        t += float(rng.exponential(1.0 / rate))
        if rng.uniform() < 0.7:
            n = int(rng.integers(fem_n[0], fem_n[1] + 1))
            ell = int(fem_ells[int(rng.integers(0, len(fem_ells)))])
            nu = float(np.exp(rng.uniform(np.log(1e-3), 0.0)))
            if make:
                p = heat_1d("fem1", n, ell, 1.0, nu, rng, True)
            else:
                rng.standard_normal(7); rng.standard_normal(16); rng.uniform(0.0, 10.0, 16)
                p = HeatProblem("fem1", n, ell, 1.0, nu, None, (np.zeros(0),) * 3,
                                np.zeros(0), np.zeros((0, 0)))
        else:
            n = int(sides[int(rng.integers(0, len(sides)))])
            ell = int(fd2_ells[int(rng.integers(0, len(fd2_ells)))])
            nu = float(np.exp(rng.uniform(np.log(1e-3), 0.0)))
            if make:
                p = heat_2d(n, ell, 0.1, nu, rng)
            else:
                rng.standard_normal((8, 8))
                p = HeatProblem("fd2", n, ell, 0.1, nu, None, (np.zeros(0),) * 3,
                                np.zeros(0), np.zeros((0, 0)))
        p.seed = seed
        yield Request(t, p)


def serving_stream(seed: int = 4, count: int = 64, rate: float = 100.0, build=True, **kw):
    """The whole stream of ``iter_serving_stream`` as a list."""
    return list(iter_serving_stream(seed, count, rate, build=build, **kw))


def dense_tridiag(t: Tridiag) -> np.ndarray:
    """Dense matrix of a (lower, diag, upper) triple (test helper)."""
    lower, diag, upper = t
    A = np.diag(diag.astype(np.float64))
    n = diag.size
    if n > 1:
        A += np.diag(lower[1:], -1) + np.diag(upper[:-1], 1)
    return A
