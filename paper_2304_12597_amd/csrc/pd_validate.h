// Host-only validation of a plan's problem and options (no HIP calls), used
// by paradiag_plan_create and paradiag_plan_check.
#pragma once

#include <cmath>
#include <string>

#include "../../include/paradiag.h"

namespace pdcheck {

inline bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Constant diagonals with equal off-diagonals.
inline bool symmetric_toeplitz(const pd_tridiag *T, int n) {
  const double d0 = T->diag[0], o0 = n > 1 ? T->upper[0] : 0.0;
  for (int i = 0; i < n; ++i)
    if (T->diag[i] != d0 || (i < n - 1 && (T->upper[i] != o0 || T->lower[i + 1] != o0)))
      return false;
  return true;
}

// Largest 1D size of a precision (the shifted-solve kernels hold one system
// per block).
inline int max_n_1d(int precision) { return precision == PD_FP64 ? 8192 : 16384; }

// Every check of plan creation that needs no device.  On failure *msg holds
// the reason.  With alpha = 1 the zero-frequency block P_0 = tau K (Section 2)
// must be nonsingular: an unpivoted float64 elimination of K whose pivot
// falls to the rounding level of the terms it is formed from (a pure-Neumann
// K leaves its last pivot at a few units of rounding) counts as singular.
// A positive scaling of K (tau, tau beta) does not change this test.
inline pd_status check_plan_args(int n, int ell, double tau, const pd_tridiag *M,
                                 const pd_tridiag *K, const pd_options &opt, std::string *msg) {
  auto fail = [msg](pd_status st, const std::string &m) {
    if (msg) *msg = m;
    return st;
  };
  if (n < 2) return fail(PD_EINVAL, "n must be at least 2");
  if (!K || !K->diag || !K->lower || !K->upper)
    return fail(PD_EINVAL, "K must provide lower, diag and upper");
  if (M && (!M->diag || !M->lower || !M->upper))
    return fail(PD_EINVAL, "M must provide lower, diag and upper (or be NULL)");
  if (opt.dims != 1 && opt.dims != 2) return fail(PD_EINVAL, "dims must be 1 or 2");
  if (opt.precision < PD_FP64 || opt.precision > PD_FP32)
    return fail(PD_EINVAL, "unknown precision");
  if (ell < 2 || ell > 4096) return fail(PD_EINVAL, "ell must lie in [2, 4096]");
  if (!is_pow2(ell)) return fail(PD_ENOTSUP, "ell must be a power of two in [2, 4096]");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(PD_EINVAL, "tau must be positive and finite");
  if (!(opt.alpha > 0.0 && opt.alpha <= 1.0)) return fail(PD_EINVAL, "alpha must lie in (0, 1]");
  if (opt.maxit < 1 || opt.maxit > 64 || opt.max_sweeps < 1 || opt.max_sweeps > 64)
    return fail(PD_EINVAL, "maxit and max_sweeps must lie in [1, 64]");
  if (opt.dims == 1) {
    const int nmax = max_n_1d(opt.precision);
    if (n > nmax)
      return fail(PD_ENOTSUP, "1D n exceeds " + std::to_string(nmax) + " for this precision");
  } else {
    if (M) return fail(PD_EINVAL, "2D plans take M = I (pass NULL)");
    if (n > 1024) return fail(PD_ENOTSUP, "2D plans need n <= 1024");
    if (!symmetric_toeplitz(K, n))
      return fail(PD_ENOTSUP, "2D plans need a symmetric Toeplitz 1D factor T");
  }
  if ((opt.krylov != PD_KRYLOV_GMRES && opt.krylov != PD_KRYLOV_FOM) || opt.fom_q < 1)
    return fail(PD_EINVAL, "unknown krylov solver or fom_q < 1");
  if (opt.shifted_solver != PD_SHIFTED_PARTITION && opt.shifted_solver != PD_SHIFTED_SINE)
    return fail(PD_EINVAL, "unknown shifted_solver");
  if (opt.bdf_order < 1 || opt.bdf_order > 6) return fail(PD_EINVAL, "bdf_order must lie in [1, 6]");
  if (opt.bdf_order > 1 &&
      (opt.precision != PD_FP64 || opt.alpha != 1.0 || opt.shifted_solver != PD_SHIFTED_PARTITION ||
       opt.early_exit != 0 || ell < 2 * opt.bdf_order))
    return fail(PD_ENOTSUP,
                "BDF plans of order > 1 need PD_FP64, alpha 1, partition solves, no "
                "early_exit and ell >= 2 * bdf_order");
  if (opt.bdf_order > 1 && opt.krylov == PD_KRYLOV_FOM && n < opt.bdf_order)
    return fail(PD_ENOTSUP, "the block Galerkin method needs n >= bdf_order");
  if (opt.shifted_solver == PD_SHIFTED_SINE) {
    if (opt.dims != 1 || opt.precision != PD_FP64 || (is_pow2(n + 1) ? n + 1 < 16 : n > 4095))
      return fail(PD_ENOTSUP,
                  "sine-basis solves need a 1D float64 plan with n + 1 a power of two >= 16 "
                  "or n <= 4095");
    if (!symmetric_toeplitz(K, n) || (M && !symmetric_toeplitz(M, n)))
      return fail(PD_ENOTSUP, "sine-basis solves need symmetric Toeplitz M and K");
  }
  for (int i = 0; i < n; ++i) {
    const double vals[6] = {K->diag[i], i > 0 ? K->lower[i] : 0.0, i < n - 1 ? K->upper[i] : 0.0,
                            M ? M->diag[i] : 1.0, (M && i > 0) ? M->lower[i] : 0.0,
                            (M && i < n - 1) ? M->upper[i] : 0.0};
    for (double v : vals)
      if (!std::isfinite(v)) return fail(PD_EINVAL, "M or K has a non-finite entry");
  }
  if (opt.alpha == 1.0 && opt.dims == 1) {
    double cprev = 0.0;
    for (int i = 0; i < n; ++i) {
      const double a = i > 0 ? K->lower[i] : 0.0, b = K->diag[i];
      const double c = i < n - 1 ? K->upper[i] : 0.0;
      const double piv = b - a * cprev;
      const double scale = std::fabs(b) + std::fabs(a * cprev);
      if (!(std::fabs(piv) > 64.0 * 2.220446049250313e-16 * scale) || !std::isfinite(piv))
        return fail(PD_ESINGULAR, "tau K is singular (zero frequency shift with alpha = 1)");
      cprev = c / piv;
    }
  }
  if (opt.alpha == 1.0 && opt.dims == 2) {
    // K_2D = I (x) T + T (x) I with symmetric Toeplitz T = tridiag(o, d, o):
    // its eigenvalues are sums of two of T's, d + 2 o cos(k pi / (n + 1)),
    // so it is singular when the smallest such sum is zero (or negative,
    // which no diffusion operator gives)
    const double d = K->diag[0], o = K->upper[0];
    const double lo = d - 2.0 * std::fabs(o) * std::cos(M_PI / (n + 1.0));
    if (!(lo > 64.0 * 2.220446049250313e-16 * (std::fabs(d) + 2.0 * std::fabs(o))))
      return fail(PD_ESINGULAR, "tau K is singular (zero frequency shift with alpha = 1)");
  }
  return PD_OK;
}

}  // namespace pdcheck
