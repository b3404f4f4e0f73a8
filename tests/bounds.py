"""Error bounds of the GPU parity tests, derived from the conditioning of
the problem (no GPU or oracle code)."""
import numpy as np

U64 = 2.0 ** -53


def tau_mu_range(p):
    """(tau mu_min, tau mu_max): extreme generalised eigenvalues of (K, M)
    times tau, from the closed forms of the uniform-grid operators (sine
    modes k = 1 and k = n; 2D: sums of two 1D eigenvalues)."""
    h = p.h
    if p.kind == "fem1":
        def mu(k):
            c = np.cos(k * np.pi * h)
            return 6.0 * p.nu / h**2 * (1 - c) / (2 + c)
    else:
        def mu(k):
            return 4.0 * p.nu / h**2 * np.sin(k * np.pi * h / 2) ** 2
    scale = 2.0 if p.dims == 2 else 1.0
    return p.tau * scale * mu(1), p.tau * scale * mu(p.n)


def capacitance_condition(p):
    """Largest eigenvalue of J_ell (its smallest is about 1): on a mode with
    tau mu = z, J_ell acts as a^ell / (a^ell - 1), a = 1 + z."""
    lo, _ = tau_mu_range(p)
    return 1.0 + 1.0 / np.expm1(p.ell * np.log1p(lo))


def fp64_error_bound(p, tol=1e-10):
    """Float64 bound on ||U - U_exact||_F / ||U_exact||_F for an
    elimination-based solve at tolerance tol: the 1e-10 bar, raised where
    the problem forces more --
      * stiffness: the shifted systems of the lowest frequencies have
        condition numbers up to about tau mu_max, and two correct
        eliminations differ by a few tens of u times that (the oracle's own
        stepping is 2.3e-9 from the exact solution on the n = 8191,
        ell = 2048 FEM workload, tau mu_max = 3.9e5);
      * the capacitance solve: GMRES stops at a residual of tol/100 ||b||,
        which the condition number of J_ell can amplify in x."""
    _, hi = tau_mu_range(p)
    stiff = 64.0 * U64 * hi
    krylov = 10.0 * (tol / 100.0) * capacitance_condition(p)
    return max(1e-10, stiff, krylov)
