// Algorithm 1 end to end, and the component entry points.
//
// One sweep (Section 2): forward time transform (first stage), shifted
// solves with the b reduction (first parfor, b = L F^{-T} e_ell), GMRES on
// the capacitance system, shifted solves of Hhat - w x (second parfor; this
// equals L - W of the paper without storing L), inverse transform.
// PD_MIXED repeats the sweep on the float64 residual (iterative refinement),
// with the residual computed in the same pass as the next forward
// transform and the correction added in the inverse transform's epilogue.
#include "pd_internal.h"

#include <algorithm>

#include <cmath>

namespace {
__global__ void negate_kernel(float *__restrict__ x, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    x[i] = -x[i];
}

// spec = -spec for a PD_MIXED plan's complex64 spectrum (spec_bytes long)
pd_status pd_negate_spectrum(pd_plan p, void *spec) {
  const size_t count = p->spec_bytes / sizeof(float);
  const size_t want = (count + 255) / 256;
  const int blocks = (int)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  hipLaunchKernelGGL(negate_kernel, dim3(blocks), dim3(256), 0, p->stream,
                     reinterpret_cast<float *>(spec), count);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}
}  // namespace

// Forward stage for 1D or 2D plans.  residual = 0: transform h from (u0, F);
// residual = 1: transform the float64 residual of (u0, F, U), with the
// partial norms left in p->red.  2D plans first apply the orthonormal DST-I
// along x (into p->wreal), so their spectra live in the DST-x domain.
pd_status pd_forward(pd_plan p, const double *u0, const double *F, const double *U, void *spec,
                     int residual) {
  if (p->dims == 1) return pd_launch_fft_forward(p, u0, F, U, spec, residual ? 1 : 0);
  pd_status st = pd_launch_dst_x(p, residual ? 1 : 0, u0, F, U, nullptr, p->wreal, 0);
  if (st != PD_OK) return st;
  return pd_launch_fft_forward(p, nullptr, p->wreal, nullptr, spec, 2);
}

int pd_forward_norm_blocks(pd_plan p) {
  return p->dims == 1 ? pd_fft_blocks(p) : pd_dst_blocks(p);
}

pd_status pd_inverse(pd_plan p, const void *spec, double *U, int accumulate) {
  if (p->dims == 1) return pd_launch_fft_inverse(p, spec, U, accumulate);
  pd_status st = pd_launch_fft_inverse(p, spec, p->wreal, 0);
  if (st != PD_OK) return st;
  return pd_launch_dst_x(p, 2, nullptr, nullptr, nullptr, p->wreal, U, accumulate);
}

namespace {

// Passes B, GMRES, C, D on the spectrum in p->spec.  has_mass: the spectrum
// already includes M (refinement residual).  accumulate: U += correction.
pd_status sweep_tail(pd_plan p, double *U, double tol, int has_mass, int accumulate,
                     pd_info *info, pd_status *gm_status) {
  const int mflag = has_mass ? 0x100 : 0;
  pd_status st = pd_launch_tridiag(p, 0 | mflag, p->spec, nullptr, nullptr);
  if (st != PD_OK) return st;
  st = pd_launch_reduce_partials(p, nullptr, p->bvec);
  if (st != PD_OK) return st;
  int its = 0;
  double rr = 0.0;
  *gm_status = pd_gmres(p, p->bvec, p->xvec, pd_gmres_tol(p->prec, tol), &its, &rr);
  if (*gm_status != PD_OK && *gm_status != PD_ENOTCONV) return *gm_status;
  st = pd_launch_tridiag(p, 1 | mflag, p->spec, p->xvec, p->spec);
  if (st != PD_OK) return st;
  st = pd_inverse(p, p->spec, U, accumulate);
  if (st != PD_OK) return st;
  if (info) {
    info->gmres_iters += its;
    info->pint_loops += its + 2;
    info->sweeps += 1;
    info->gmres_rel_residual = rr;
  }
  return PD_OK;
}

// One sweep with the whole tail enqueued ahead: the capacitance GMRES runs
// as many iterations as the plan's last solve needed (later ones return at
// once after convergence), then x = V y, pass C and pass D, all before the
// single synchronisation.  If GMRES had not converged by then, it continues
// from its state, and pass A (whose spectrum pass C overwrote) and passes C,
// D are redone.
pd_status solve_speculative(pd_plan p, const double *u0, const double *F, double *U, double tol,
                            pd_info *info) {
  const double rtol = pd_gmres_tol(p->prec, tol);
  pd_status st;
  {
    PdRange r("paradiag: pass B (shifted solves, b)");
    st = pd_launch_tridiag(p, 0, p->spec, nullptr, nullptr);
    if (st != PD_OK) return st;
    st = pd_launch_reduce_partials(p, nullptr, p->bvec);
    if (st != PD_OK) return st;
  }
  const int pred = p->gm_pred < 1 ? 1 : (p->gm_pred > p->maxit ? p->maxit : p->gm_pred);
  {
    PdRange r("paradiag: capacitance GMRES (enqueued ahead)");
    st = pd_gmres_enqueue(p, p->bvec, p->xvec, rtol, pred);
    if (st != PD_OK) return st;
  }
  {
    PdRange r("paradiag: pass C (shifted solves)");
    st = pd_launch_tridiag(p, 1, p->spec, p->xvec, p->spec);
    if (st != PD_OK) return st;
  }
  {
    PdRange r("paradiag: pass D (inverse transform)");
    st = pd_inverse(p, p->spec, U, 0);
    if (st != PD_OK) return st;
  }
  {
    PdRange r("paradiag: wait for the solve");
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  }
  int m;
  double res, beta;
  bool done;
  pd_gmres_read(p, &m, &res, &beta, &done);
  if (!std::isfinite(beta)) {
    pd_set_error("capacitance right-hand side is not finite");
    return PD_ENONFINITE;
  }
  if (!std::isfinite(res)) {
    pd_set_error("capacitance GMRES produced a non-finite residual");
    return PD_ENONFINITE;
  }
  pd_status gst = PD_OK;
  if (!done && m < p->maxit) {
    int its = m;
    double rr = 0.0;
    gst = pd_gmres_continue(p, p->xvec, rtol, &its, &rr);
    if (gst != PD_OK && gst != PD_ENOTCONV) return gst;
    st = pd_forward(p, u0, F, nullptr, p->spec, 0);
    if (st != PD_OK) return st;
    st = pd_launch_tridiag(p, 1, p->spec, p->xvec, p->spec);
    if (st != PD_OK) return st;
    st = pd_inverse(p, p->spec, U, 0);
    if (st != PD_OK) return st;
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
    pd_gmres_read(p, &m, &res, &beta, &done);
  } else if (!done) {
    gst = PD_ENOTCONV;
  }
  if (m > 0) p->gm_pred = m;
  p->gm_seen = 1;
  if (info) {
    info->gmres_iters = m;
    info->pint_loops = m + 2;
    info->sweeps = 1;
    info->gmres_rel_residual = beta > 0.0 ? res / beta : 0.0;
  }
  if (p->check_residual) {
    double rel, est;
    st = pd_residual_impl(p, u0, F, U, &rel, &est);
    if (st != PD_OK) return st;
    if (info) {
      info->rel_residual = rel;
      info->est_rel_error = est;
    }
  }
  if (gst == PD_ENOTCONV) pd_set_error("tolerance not reached");
  return gst;
}

// Sine-basis form: DST-I of every time row of h (into the spectrum buffer,
// read as [ell][n] float64), the per-mode time transform and solve (into U),
// DST-I of every row of U in place.  The capacitance system is diagonal in
// this basis and solved exactly, so no Krylov iteration runs.
pd_status solve_sine(pd_plan p, const double *u0, const double *F, double *U, pd_info *info) {
  double *A = reinterpret_cast<double *>(p->spec);
  pd_status st = pd_launch_sine_dst(p, 0, u0, F, nullptr, A);
  if (st != PD_OK) return st;
  st = pd_launch_sine_modal(p, A, U);
  if (st != PD_OK) return st;
  st = pd_launch_sine_dst(p, 1, nullptr, nullptr, U, U);
  if (st != PD_OK) return st;
  if (info) {
    info->gmres_iters = 0;
    info->pint_loops = 1;
    info->sweeps = 1;
    info->gmres_rel_residual = 0.0;
  }
  if (p->check_residual) {
    double rel, est;
    st = pd_residual_impl(p, u0, F, U, &rel, &est);
    if (st != PD_OK) return st;
    if (info) {
      info->rel_residual = rel;
      info->est_rel_error = est;
    }
  }
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  return PD_OK;
}

// Algorithm 1 with Algorithm 2 for the capacitance system: pass B, the
// projection method (its residual check every fom_q steps is one parfor),
// pass C, pass D.  #PinT = checks + 2 (Section 3).
pd_status solve_fom(pd_plan p, const double *u0, const double *F, double *U, double tol,
                    pd_info *info) {
  pd_status st = pd_launch_tridiag(p, 0, p->spec, nullptr, nullptr);
  if (st != PD_OK) return st;
  st = pd_launch_reduce_partials(p, nullptr, p->bvec);
  if (st != PD_OK) return st;
  int m = 0, checks = 0;
  double rr = 0.0;
  const pd_status fst = pd_fom(p, p->bvec, p->xvec, tol * PD_GMRES_TOL_FACTOR, &m, &rr, &checks);
  if (fst != PD_OK && fst != PD_ENOTCONV) return fst;
  st = pd_launch_tridiag(p, 1, p->spec, p->xvec, p->spec);
  if (st != PD_OK) return st;
  st = pd_inverse(p, p->spec, U, 0);
  if (st != PD_OK) return st;
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  if (info) {
    info->gmres_iters = m;
    info->pint_loops = checks + 2;
    info->sweeps = 1;
    info->gmres_rel_residual = rr;
  }
  if (p->check_residual) {
    double rel, est;
    st = pd_residual_impl(p, u0, F, U, &rel, &est);
    if (st != PD_OK) return st;
    if (info) {
      info->rel_residual = rel;
      info->est_rel_error = est;
    }
  }
  if (fst == PD_ENOTCONV) pd_set_error("Algorithm 2 did not reach the tolerance");
  return fst;
}

bool check_ptrs(const void *a, const void *b, const void *c) {
  if (!a || !b || !c) {
    pd_set_error("NULL array argument");
    return false;
  }
  return true;
}

}  // namespace

extern "C" pd_status paradiag_solve(pd_plan p, const double *u0, const double *F, double *U,
                                    double tol, pd_info *info) {
  if (!p) {
    pd_set_error("plan is NULL");
    return PD_EINVAL;
  }
  if (!check_ptrs(u0, F, U)) return PD_EINVAL;
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    pd_set_error("tol must be positive and finite");
    return PD_EINVAL;
  }
  if (info) {
    info->gmres_iters = 0;
    info->sweeps = 0;
    info->pint_loops = 0;
    info->rel_residual = -1.0;
    info->gmres_rel_residual = -1.0;
    info->early_exit = 0;
    info->est_rel_error = -1.0;
  }
  PdRange whole("paradiag_solve");
  pd_status gst = PD_OK;
  if (p->bdf_s > 1) return pd_bdf_solve(p, u0, F, U, tol, info);
  if (p->sine) return solve_sine(p, u0, F, U, info);
  pd_status st;
  {
    PdRange r("paradiag: pass A (forward transform)");
    st = pd_forward(p, u0, F, nullptr, p->spec, 0);
    if (st != PD_OK) return st;
  }
  if (p->early_exit) {
    // Algorithm 3: U_1 = P^{-1} Ghat F^{-T} D_alpha^{-1} (pass C with x = 0,
    // pass D), accepted when its residual in the original all-at-once system
    // is at most tol * ||M U_1||_F (the paper's ||U_1||_F when M = I; with a
    // mass matrix every residual row carries M)
    PD_HIP_CHECK(hipMemsetAsync(p->xvec, 0, sizeof(double) * (size_t)p->nbar, p->stream));
    st = pd_launch_tridiag(p, 1, p->spec, p->xvec, p->spec);
    if (st != PD_OK) return st;
    st = pd_inverse(p, p->spec, U, 0);
    if (st != PD_OK) return st;
    double rn2, gn2, un2;
    st = pd_residual_norms(p, u0, F, U, &rn2, &gn2, &un2);
    if (st != PD_OK) return st;
    if (std::sqrt(rn2) <= tol * std::sqrt(un2)) {
      if (info) {
        info->early_exit = 1;
        info->pint_loops = 1;
        info->rel_residual = gn2 > 0.0 ? std::sqrt(rn2 / gn2) : std::sqrt(rn2);
      }
      return PD_OK;
    }
    // rejected: the spectrum (overwritten by pass C) is formed again and the
    // full method runs
    st = pd_forward(p, u0, F, nullptr, p->spec, 0);
    if (st != PD_OK) return st;
  }
  if (p->krylov == PD_KRYLOV_FOM) return solve_fom(p, u0, F, U, tol, info);
  if (p->prec != PD_MIXED && pd_gmres_fused_ok(p)) return solve_speculative(p, u0, F, U, tol, info);
  st = sweep_tail(p, U, tol, 0, 0, info, &gst);
  if (st != PD_OK) return st;
  pd_status final_status = gst;
  if (p->prec == PD_MIXED) {
    double rel = -1.0, prev = -1.0;
    bool converged = false, stalled = false;
    int swaps = 0;
    for (int s = 1; s < p->max_sweeps; ++s) {
      PdRange r("paradiag: refinement sweep");
      // residual of the current iterate, fused with the next forward
      // transform, into the other spectrum buffer: the last correction's
      // spectrum stays in p->spec2
      std::swap(p->spec, p->spec2);
      ++swaps;
      st = pd_forward(p, u0, F, U, p->spec, 1);
      if (st != PD_OK) return st;
      double rn2, gn2;
      st = pd_sum_norms(p, pd_forward_norm_blocks(p), &rn2, &gn2);
      if (st != PD_OK) return st;
      if (!std::isfinite(rn2) || !std::isfinite(gn2)) {
        pd_set_error("non-finite residual during refinement");
        return PD_ENONFINITE;
      }
      rel = gn2 > 0.0 ? std::sqrt(rn2 / gn2) : std::sqrt(rn2);
      if (rel <= tol) {
        converged = true;
        break;
      }
      if (prev >= 0.0 && rel >= prev) {
        // stalled: the last correction did not lower the residual.  Take it
        // back (U -= its inverse transform, from the negated spectrum) so
        // that the best iterate is returned, and stop.
        st = pd_negate_spectrum(p, p->spec2);
        if (st != PD_OK) return st;
        st = pd_inverse(p, p->spec2, U, 1);
        if (st != PD_OK) return st;
        rel = prev;
        stalled = true;
        break;
      }
      prev = rel;
      st = sweep_tail(p, U, tol, 1, 1, info, &gst);
      if (st != PD_OK) return st;
      rel = -1.0;
    }
    if (swaps & 1) std::swap(p->spec, p->spec2);
    if (stalled) pd_set_error("refinement stalled: the residual stopped falling");
    const bool checked = rel >= 0.0;   // the loop's last check is of this U
    if (!checked || p->check_residual) {
      // the standalone residual: the stopping test after the last sweep, or
      // the accuracy report (with the error bound) when it was asked for
      double r2, est;
      st = pd_residual_impl(p, u0, F, U, &r2, &est);
      if (st != PD_OK) return st;
      if (!checked) {
        rel = r2;
        converged = rel <= tol;
      }
      if (info) info->est_rel_error = est;
    }
    if (info) info->rel_residual = rel;
    final_status = converged ? PD_OK : PD_ENOTCONV;
    if (final_status == PD_ENOTCONV && stalled) {
      PD_HIP_CHECK(hipStreamSynchronize(p->stream));
      return final_status;
    }
  } else {
    if (p->check_residual) {
      double rel, est;
      st = pd_residual_impl(p, u0, F, U, &rel, &est);
      if (st != PD_OK) return st;
      if (info) {
        info->rel_residual = rel;
        info->est_rel_error = est;
      }
    }
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  }
  if (final_status == PD_ENOTCONV) pd_set_error("tolerance not reached");
  return final_status;
}

extern "C" pd_status paradiag_solve_batch(const pd_plan *plans, int count, const double *const *u0,
                                          const double *const *F, double *const *U, double tol,
                                          pd_info *infos) {
  if (!plans || count < 0 || (count > 0 && (!u0 || !F || !U))) {
    pd_set_error("invalid batch arguments");
    return PD_EINVAL;
  }
  if (count == 0) return PD_OK;
  PdRange whole("paradiag_solve_batch");
  for (int i = 0; i < count; ++i)
    if (!plans[i] || !u0[i] || !F[i] || !U[i]) {
      pd_set_error("invalid batch arguments");
      return PD_EINVAL;
    }
  if (!(tol > 0.0) || !std::isfinite(tol)) {
    pd_set_error("tol must be positive and finite");
    return PD_EINVAL;
  }
  if (pd_batchable(plans, count)) return pd_solve_batch_impl(plans, count, u0, F, U, tol, infos);
  // Split into groups that batch together (1D, uniform, same precision and
  // iteration limit; see pd_batchable), each solved in one submission; the
  // rest (2D, mixed precision, non-uniform grids, BDF, the sine basis,
  // Algorithm 2, repeated plans) one after another.
  std::vector<int> rest;
  std::vector<std::vector<int>> groups;
  for (int i = 0; i < count; ++i) {
    bool placed = false;
    if (pd_batchable(&plans[i], 1)) {
      for (auto &g : groups) {
        std::vector<pd_plan> trial;
        trial.push_back(plans[g[0]]);
        trial.push_back(plans[i]);
        bool dup = false;
        for (int j : g) dup = dup || plans[j] == plans[i];
        if (!dup && pd_batchable(trial.data(), 2)) {
          g.push_back(i);
          placed = true;
          break;
        }
      }
      if (!placed) {
        groups.push_back({i});
        placed = true;
      }
    }
    if (!placed) rest.push_back(i);
  }
  pd_status worst = PD_OK;
  for (const auto &g : groups) {
    if (g.size() == 1) {
      rest.push_back(g[0]);
      continue;
    }
    std::vector<pd_plan> gp;
    std::vector<const double *> gu, gf;
    std::vector<double *> gU;
    std::vector<pd_info> gi(g.size());
    for (int i : g) {
      gp.push_back(plans[i]);
      gu.push_back(u0[i]);
      gf.push_back(F[i]);
      gU.push_back(U[i]);
    }
    const pd_status st = pd_solve_batch_impl(gp.data(), (int)g.size(), gu.data(), gf.data(),
                                             gU.data(), tol, infos ? gi.data() : nullptr);
    if (st != PD_OK && st != PD_ENOTCONV) return st;
    if (st == PD_ENOTCONV) worst = PD_ENOTCONV;
    if (infos)
      for (size_t t = 0; t < g.size(); ++t) infos[g[t]] = gi[t];
  }
  std::sort(rest.begin(), rest.end());
  for (int i : rest) {
    pd_status st = paradiag_solve(plans[i], u0[i], F[i], U[i], tol, infos ? &infos[i] : nullptr);
    if (st != PD_OK && st != PD_ENOTCONV) return st;
    if (st == PD_ENOTCONV) worst = PD_ENOTCONV;
  }
  return worst;
}

extern "C" pd_status paradiag_forward_transform(pd_plan p, const double *u0, const double *F,
                                                void *Hhat) {
  if (!p) {
    pd_set_error("plan is NULL");
    return PD_EINVAL;
  }
  if (!check_ptrs(u0, F, Hhat)) return PD_EINVAL;
  if (p->bdf_s > 1) {
    pd_status st = pd_bdf_rhs(p, u0, F, p->dims == 2 ? p->bdf_h : p->wreal);
    if (st != PD_OK) return st;
    if (p->dims == 2) {
      st = pd_launch_dst_x_rows(p, p->bdf_h, p->wreal, p->ell, 0);
      if (st != PD_OK) return st;
    }
    return pd_launch_fft_forward(p, nullptr, p->wreal, nullptr, Hhat, 2);
  }
  return pd_forward(p, u0, F, nullptr, Hhat, 0);
}

extern "C" pd_status paradiag_shifted_solve(pd_plan p, const void *Hhat, const double *x,
                                            void *Uhat, double *b) {
  if (!p || !Hhat || (!Uhat && !b)) {
    pd_set_error("invalid shifted-solve arguments");
    return PD_EINVAL;
  }
  if (p->bdf_s > 1 && (b || x)) {
    pd_set_error("BDF plans: the shifted solves take x = NULL and produce Uhat only");
    return PD_ENOTSUP;
  }
  pd_status st;
  if (b) {
    st = pd_launch_tridiag(p, 0, Hhat, nullptr, nullptr);
    if (st != PD_OK) return st;
    st = pd_launch_reduce_partials(p, nullptr, b);
    if (st != PD_OK) return st;
  }
  if (Uhat) {
    st = pd_launch_tridiag(p, 1, Hhat, x, Uhat);
    if (st != PD_OK) return st;
  }
  return PD_OK;
}

extern "C" pd_status paradiag_capacitance_apply(pd_plan p, const double *v, double *Jv) {
  if (!p || !v || !Jv) {
    pd_set_error("invalid capacitance arguments");
    return PD_EINVAL;
  }
  return pd_capacitance_apply_impl(p, v, Jv);
}

extern "C" pd_status paradiag_capacitance_solve(pd_plan p, const double *b, double *x, double rtol,
                                                int *iters, double *relres) {
  if (!p || !b || !x || !(rtol > 0.0)) {
    pd_set_error("invalid capacitance-solve arguments");
    return PD_EINVAL;
  }
  pd_status st = pd_gmres(p, b, x, rtol, iters, relres);
  if (st != PD_OK && st != PD_ENOTCONV) return st;
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  if (st == PD_ENOTCONV) pd_set_error("capacitance GMRES did not reach rtol");
  return st;
}

extern "C" pd_status paradiag_inverse_transform(pd_plan p, const void *Uhat, double *U) {
  if (!p || !Uhat || !U) {
    pd_set_error("invalid inverse-transform arguments");
    return PD_EINVAL;
  }
  return pd_inverse(p, Uhat, U, 0);
}

extern "C" pd_status paradiag_residual(pd_plan p, const double *u0, const double *F,
                                       const double *U, double *rel) {
  if (!p || !rel) {
    pd_set_error("invalid residual arguments");
    return PD_EINVAL;
  }
  if (!check_ptrs(u0, F, U)) return PD_EINVAL;
  if (p->bdf_s > 1) {
    double rn2, gn2;
    pd_status st = pd_bdf_residual_norms(p, u0, F, U, &rn2, &gn2);
    if (st != PD_OK) return st;
    *rel = gn2 > 0.0 ? std::sqrt(rn2 / gn2) : std::sqrt(rn2);
    return PD_OK;
  }
  return pd_residual_impl(p, u0, F, U, rel);
}

extern "C" pd_status paradiag_sine_transform(pd_plan p, const double *in, double *out) {
  if (!p || !in || !out) {
    pd_set_error("invalid sine-transform arguments");
    return PD_EINVAL;
  }
  if (!p->sine) {
    pd_set_error("the plan was not created with PD_SHIFTED_SINE");
    return PD_ENOTSUP;
  }
  return pd_launch_sine_dst(p, 1, nullptr, nullptr, in, out);
}
