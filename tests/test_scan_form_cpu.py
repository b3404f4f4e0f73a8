"""CPU replica of the recurrence-form shifted solve (csrc/pd_scan.h), in
float64 numpy, against a dense solve of the same symmetric Toeplitz
tridiagonal system (the shifted systems lambda_k M + tau K of Section 2 on
uniform grids).

The replica restates the kernel's steps in its order: the per-chunk forward
recurrence, the scan of the chunk maps x -> R x + e across the group (lanes
in waves of 64, the waves' totals combined in order), the chunk's share of
z_0 from a Horner sum, the Sherman-Morrison correction of the corner term
folded into the forward values, the backward recurrence and its scan, and
the final scaling by 1/kappa.  The per-frequency constants are built as the
host builds them (long double there, float64 here).
"""
import numpy as np
import pytest


def table(a, b, n, MR, real):
    """kappa, r (symmetric: r1 = r2), beta, K = sum_{q<MR} r^(2q+1)."""
    if real:
        disc = max(b.real * b.real - 4 * a.real * a.real, 0.0)
        s = np.sqrt(disc)
        kap = complex((b.real + s) / 2 if b.real >= 0 else (b.real - s) / 2)
    else:
        s = np.sqrt(b * b - 4 * a * a + 0j)
        k1, k2 = (b + s) / 2, (b - s) / 2
        kap = k1 if abs(k1) >= abs(k2) else k2
    r = -a / kap
    rho = r * r
    w0 = np.sum(rho ** np.arange(n))
    beta = rho / (1 + rho * w0)
    K = np.sum(r ** (2 * np.arange(MR) + 1))
    return kap, r, beta, K


def _pattern(lane, shift, rowmask):
    """Source lane (in the same wave) and validity of a DPP move: row shift
    right (shift > 0) or left (< 0) within rows of 16 lanes, or the row
    broadcasts of lane 15 / lane 31 ("b15", "b31") into the rows of rowmask."""
    base = lane - lane % 64
    w = lane % 64
    row, i = w // 16, w % 16
    if shift == "b15":
        ok = (row > 0) & (((rowmask >> row) & 1) == 1)
        return base + np.maximum(row * 16 - 1, 0), ok
    if shift == "b31":
        ok = ((rowmask >> row) & 1) == 1
        return base + 31, ok
    if shift > 0:
        ok = i >= shift
        return base + np.where(ok, w - shift, w), ok
    ok = i - shift < 16
    return base + np.where(ok, w - shift, w), ok


def scan_solve(y, a, b, P, MR, real=False):
    n = y.size
    kap, r, beta, K_full = table(a, b, n, MR, real)
    N = P * MR
    d = np.zeros(N, complex)
    d[:n] = y
    d = d.reshape(P, MR)
    lt = np.arange(P)
    length = np.clip(n - lt * MR, 0, MR)
    lane, wv = lt % 64, lt // 64
    W = min(P, 64)            # shuffle width: one wave, or the group if smaller
    NW = max(P // 64, 1)
    R = r ** MR
    # forward recurrence inside each chunk, from zero
    acc = np.zeros(P, complex)
    for q in range(MR):
        acc = d[:, q] + r * acc
        d[:, q] = acc
    # scan of the chunk maps across each wave: for whole waves by rows of 16
    # lanes, then the rows' last lanes (the kernel's DPP row shifts and row
    # broadcasts); for smaller groups by Hillis-Steele steps of width P
    c, m = acc.copy(), np.full(P, R)
    if W == 64:
        for shift, rows in ((1, 15), (2, 15), (4, 15), (8, 15), ("b15", 10), ("b31", 12)):
            src, ok = _pattern(lt, shift, rows)
            oc, om = np.where(ok, c[src], 0), np.where(ok, m[src], 1)
            c, m = c + m * oc, m * om
    else:
        s = 1
        while s < W:
            oc, om = np.roll(c, s), np.roll(m, s)
            inn = (lane % W) >= s
            c, m = np.where(inn, c + m * oc, c), np.where(inn, m * om, m)
            s *= 2
    ex = np.where(lane % W > 0, np.roll(c, 1), 0)
    pl = np.where(lane % W > 0, np.roll(m, 1), 1)           # R^lane
    R64 = R ** W
    tot = c.reshape(NW, -1)[:, -1]                           # waves' totals
    C = np.zeros(NW, complex)
    for w in range(1, NW):
        C[w] = tot[w - 1] + R64 * C[w - 1]
    ex = ex + pl * C[wv]
    a0 = pl * R64 ** wv                                      # r^(lt MR)
    # this chunk's share of z_0 = sum_i r^i v_i
    h = np.zeros(P, complex)
    Kt = np.zeros(P, complex)
    for q in range(MR - 1, -1, -1):
        h = np.where(q < length, d[:, q] + r * h, h)
    for q in range(MR):
        Kt = np.where(q < length, Kt + r ** (2 * q + 1), Kt)
    assert np.allclose(Kt[length == MR], K_full)
    z0 = np.sum(a0 * (h + ex * Kt))
    # corrected forward values u_q + r^q (r ex - beta z_0 r^s0)
    E = r * ex - beta * z0 * a0
    for q in range(MR):
        d[:, q] = np.where(q < length, d[:, q] + r ** q * E, 0)
    # backward recurrence and its scan from the right
    acc = np.zeros(P, complex)
    for q in range(MR - 1, -1, -1):
        acc = d[:, q] + r * acc
        d[:, q] = acc
    cz, m = acc.copy(), np.full(P, R)
    if W == 64:
        # rows of 16 from the right, then rows 0 and 2 take the next row's
        # first lane, then rows 0 and 1 take lane 32
        for shift in (-1, -2, -4, -8):
            src, ok = _pattern(lt, shift, 15)
            oz, om = np.where(ok, cz[src], 0), np.where(ok, m[src], 1)
            cz, m = cz + m * oz, m * om
        base = (lt // 64) * 64
        src = base + (((lane | 15) + 1) & 63)
        inn = ((lane >> 4) & 1) == 0
        cz, m = np.where(inn, cz + m * cz[src], cz), np.where(inn, m * m[src], m)
        src = base + 32
        inn = lane < 32
        cz, m = np.where(inn, cz + m * cz[src], cz), np.where(inn, m * m[src], m)
    else:
        s = 1
        while s < W:
            oz, om = np.roll(cz, -s), np.roll(m, -s)
            inn = (lane % W) + s < W
            cz, m = np.where(inn, cz + m * oz, cz), np.where(inn, m * om, m)
            s *= 2
    exz = np.where(lane % W < W - 1, np.roll(cz, -1), 0)
    pr = np.where(lane % W < W - 1, np.roll(m, -1), 1)       # R^(W-1-lane)
    tot = cz.reshape(NW, -1)[:, 0]
    CZ = np.zeros(NW, complex)
    for w in range(NW - 2, -1, -1):
        CZ[w] = tot[w + 1] + R64 * CZ[w + 1]
    exz = exz + pr * CZ[wv]
    for q in range(MR):
        d[:, q] = (d[:, q] + r ** (MR - q) * exz) / kap
    return d.reshape(N)[:n]


def dense(y, a, b):
    n = y.size
    A = np.diag(np.full(n, b)) + np.diag(np.full(n - 1, a), 1) + np.diag(np.full(n - 1, a), -1)
    return np.linalg.solve(A, y)


def heat_shift(kind, n, ell, k, nu=1.0):
    """Diagonals of lambda_k M + tau K, 1D FD (M = I) or P1 FEM, (0, 1)."""
    h, tau = 1.0 / (n + 1), 1.0 / ell
    lam = 1 - np.exp(-2j * np.pi * k / ell)
    if k == 0 or 2 * k == ell:
        lam = complex(lam.real, 0.0)
    if kind == "fd":
        m0, m1, k0, k1 = 1.0, 0.0, 2 * nu / h ** 2, -nu / h ** 2
    else:
        m0, m1, k0, k1 = 4 * h / 6, h / 6, 2 * nu / h, -nu / h
    return lam * m1 + tau * k1, lam * m0 + tau * k0, lam.imag == 0


@pytest.mark.parametrize("kind,n,ell,P,MR", [
    ("fem", 1000, 64, 128, 8), ("fd", 511, 256, 64, 8), ("fd", 255, 64, 32, 8),
    ("fem", 127, 32, 16, 8), ("fd", 4095, 1024, 512, 8), ("fem", 2047, 128, 128, 16),
    ("fd", 64 * 8 - 9, 16, 64, 8), ("fem", 130, 16, 64, 4)])
def test_scan_form_matches_dense(kind, n, ell, P, MR):
    rng = np.random.default_rng(n + ell)
    for k in (0, 1, 2, ell // 4, ell // 2):
        a, b, real = heat_shift(kind, n, ell, k)
        y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x = scan_solve(y, a, b, P, MR, real)
        xd = dense(y, a, b)
        # the matrix is normal (diagonalised by the real sine basis), so its
        # condition number is the ratio of its eigenvalues' moduli
        ev = np.abs(b + 2 * a * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
        cond = ev.max() / ev.min()
        err = np.linalg.norm(x - xd) / np.linalg.norm(xd)
        assert err < 1e-14 * max(cond, 10.0), (k, err, cond)


def test_scan_form_identity_pins():
    """kappa (1 + r^2) = b, and the factored form plus the corner term
    reproduces the matrix (the identity the solve rests on)."""
    for kind, n, ell in (("fem", 50, 32), ("fd", 40, 16)):
        for k in range(ell // 2 + 1):
            a, b, real = heat_shift(kind, n, ell, k)
            kap, r, beta, _ = table(a, b, n, 8, real)
            assert abs(kap * (1 + r * r) - b) <= 1e-13 * abs(b)
            Z = np.diag(np.ones(n - 1), -1)
            I = np.eye(n)
            Pm = kap * (I - r * Z) @ (I - r * Z.T)
            Pm[0, 0] += kap * r * r
            A = np.diag(np.full(n, b)) + np.diag(np.full(n - 1, a), 1) + np.diag(np.full(n - 1, a), -1)
            assert np.max(np.abs(Pm - A)) <= 1e-12 * np.max(np.abs(A))
            assert abs(r) <= 1 + 1e-12
