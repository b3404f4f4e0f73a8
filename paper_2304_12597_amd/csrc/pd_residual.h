// float64 all-at-once residual at one space-time point (device helper shared
// by the fused refinement transform and the standalone residual kernel).
#pragma once
#include "pd_internal.h"

// tau T's diagonals for the 2D stencil: constant on uniform grids (uni),
// then no coefficient loads per point
struct Stencil2 {
  int uni;
  double kl, kd, ku;
};

// The 2D residual at point (x, y) of time row t (i = y n + x) for callers
// that walk x and y: the same expressions as residual_point's 2D branch, with
// tau T's diagonals from the scalars when uniform (the boundary entries they
// would differ in are never used).
static __device__ __forceinline__ void residual_point_2d(int t, int x, int y, int n, int nbar,
                                                  double tau, const double *__restrict__ u0,
                                                  const double *__restrict__ F,
                                                  const double *__restrict__ U,
                                                  const double *__restrict__ coef,
                                                  const Stencil2 &sk, double &r_out,
                                                  double &g_out) {
  const int i = y * n + x;
  const double *Ft = F + (size_t)t * nbar;
  const double *Ut = U + (size_t)t * nbar;
  double h = tau * Ft[i];
  if (t == 0) h += u0[i];
  double z = h - Ut[i];
  if (t > 0) z += U[(size_t)(t - 1) * nbar + i];
  double kdx, kdy, klx, kux, kly, kuy;
  if (sk.uni) {
    kdx = kdy = sk.kd;
    klx = kly = sk.kl;
    kux = kuy = sk.ku;
  } else {
    const double *KL = coef + 3 * n, *KD = coef + 4 * n, *KU = coef + 5 * n;
    kdx = KD[x]; kdy = KD[y]; klx = KL[x]; kux = KU[x]; kly = KL[y]; kuy = KU[y];
  }
  double ku = (kdx + kdy) * Ut[i];
  if (x > 0) ku += klx * Ut[i - 1];
  if (x < n - 1) ku += kux * Ut[i + 1];
  if (y > 0) ku += kly * Ut[i - n];
  if (y < n - 1) ku += kuy * Ut[i + n];
  r_out = z - ku;
  g_out = h;
}

// float64 all-at-once residual R_t = G_t - ((M + tau K) u_t - M u_{t-1}) at
// one space-time point, with G_t = M h_t, h_t = tau f_t (+ u0 at t = 0).
// coef rows: ML MD MU tKL tKD tKU (tK = tau K; 2D: the 1D factor tau T).
static __device__ __forceinline__ void residual_point(int t, int i, int n, int nbar, int dims,
                                               double tau, const double *__restrict__ u0,
                                               const double *__restrict__ F,
                                               const double *__restrict__ U,
                                               const double *__restrict__ coef,
                                               double &r_out, double &g_out) {
  const double *Ft = F + (size_t)t * nbar;
  const double *Ut = U + (size_t)t * nbar;
  const double *Up = t > 0 ? U + (size_t)(t - 1) * nbar : nullptr;
  auto h_at = [&](int j) {
    double h = tau * Ft[j];
    if (t == 0) h += u0[j];
    return h;
  };
  auto z_at = [&](int j) {  // h - u_t + u_{t-1}
    double z = h_at(j) - Ut[j];
    if (Up) z += Up[j];
    return z;
  };
  if (dims == 1) {
    const double ML = coef[i], MD = coef[n + i], MU = coef[2 * n + i];
    const double KL = coef[3 * n + i], KD = coef[4 * n + i], KU = coef[5 * n + i];
    double g = MD * h_at(i);
    double r = MD * z_at(i) - KD * Ut[i];
    if (i > 0) {
      g += ML * h_at(i - 1);
      r += ML * z_at(i - 1) - KL * Ut[i - 1];
    }
    if (i < n - 1) {
      g += MU * h_at(i + 1);
      r += MU * z_at(i + 1) - KU * Ut[i + 1];
    }
    r_out = r;
    g_out = g;
  } else {
    const int y = i / n, x = i - y * n;
    const double *KL = coef + 3 * n, *KD = coef + 4 * n, *KU = coef + 5 * n;
    double g = h_at(i);
    double ku = (KD[x] + KD[y]) * Ut[i];
    if (x > 0) ku += KL[x] * Ut[i - 1];
    if (x < n - 1) ku += KU[x] * Ut[i + 1];
    if (y > 0) ku += KL[y] * Ut[i - n];
    if (y < n - 1) ku += KU[y] * Ut[i + n];
    r_out = z_at(i) - ku;
    g_out = g;
  }
}

