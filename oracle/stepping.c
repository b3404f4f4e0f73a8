/*
 * ORACLE -- test infrastructure only.  Nothing in the product path may link,
 * load or call this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark do.
 *
 * Plain sequential backward-Euler time stepping for the 1D all-at-once
 * system of Section 1 (the matrix equation with Sigma_1, generalised with a
 * mass matrix M):
 *
 *     (M + tau K) u_j = M (u_{j-1} + tau f_j),   j = 1..ell,
 *
 * which is exactly the block-forward-substitution of that lower block
 * bidiagonal system.  M + tau K is a real symmetric positive definite
 * tridiagonal matrix for every heat problem here, so the Thomas algorithm
 * without pivoting is used; it is factored once and reused for every step.
 *
 * Layout: tridiagonals are three length-n arrays (lower[i] multiplies
 * x[i-1], upper[i] multiplies x[i+1]); Ml == NULL means M = I.  F and U are
 * time-major [ell][n], row j holding time t_{j+1}.  Returns 0 on success,
 * 1 on a zero pivot, 2 on bad sizes or allocation failure.
 */
#include <stdlib.h>
#include <string.h>

static void mass_apply(int n, const double *Ml, const double *Md,
                       const double *Mu, const double *v, double *out)
{
    for (int i = 0; i < n; ++i) {
        if (!Md) { out[i] = v[i]; continue; }
        double s = Md[i] * v[i];
        if (i > 0) s += Ml[i] * v[i - 1];
        if (i < n - 1) s += Mu[i] * v[i + 1];
        out[i] = s;
    }
}

int pd_oracle_step_1d(int n, int ell, double tau,
                      const double *Ml, const double *Md, const double *Mu,
                      const double *Kl, const double *Kd, const double *Ku,
                      const double *u0, const double *F, double *U)
{
    if (n < 1 || ell < 1) return 2;
    double *cp = (double *)malloc(sizeof(double) * n);   /* c'_i        */
    double *ip = (double *)malloc(sizeof(double) * n);   /* 1 / pivot_i */
    double *lo = (double *)malloc(sizeof(double) * n);   /* A lower     */
    double *w = (double *)malloc(sizeof(double) * n);
    double *rhs = (double *)malloc(sizeof(double) * n);
    if (!cp || !ip || !lo || !w || !rhs) {
        free(cp); free(ip); free(lo); free(w); free(rhs);
        return 2;
    }
    /* A = M + tau K, Thomas factorisation. */
    for (int i = 0; i < n; ++i) {
        double a = (i > 0) ? (Md ? Ml[i] : 0.0) + tau * Kl[i] : 0.0;
        double b = (Md ? Md[i] : 1.0) + tau * Kd[i];
        double c = (i < n - 1) ? (Md ? Mu[i] : 0.0) + tau * Ku[i] : 0.0;
        double piv = b - ((i > 0) ? a * cp[i - 1] : 0.0);
        if (piv == 0.0) {
            free(cp); free(ip); free(lo); free(w); free(rhs);
            return 1;
        }
        lo[i] = a;
        ip[i] = 1.0 / piv;
        cp[i] = c * ip[i];
    }
    const double *prev = u0;
    for (int j = 0; j < ell; ++j) {
        const double *f = F + (size_t)j * n;
        for (int i = 0; i < n; ++i) w[i] = prev[i] + tau * f[i];
        mass_apply(n, Ml, Md, Mu, w, rhs);
        double *u = U + (size_t)j * n;
        /* forward substitution */
        for (int i = 0; i < n; ++i) {
            double d = rhs[i] - ((i > 0) ? lo[i] * u[i - 1] : 0.0);
            u[i] = d * ip[i];
        }
        /* back substitution */
        for (int i = n - 2; i >= 0; --i) u[i] -= cp[i] * u[i + 1];
        prev = u;
    }
    free(cp); free(ip); free(lo); free(w); free(rhs);
    return 0;
}
