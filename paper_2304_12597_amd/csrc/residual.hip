// Standalone float64 residual of the all-at-once system,
// ||G - A(U)||_F / ||G||_F (Algorithm 3, the residual test on U_1; here the
// accuracy report of a solve and the stopping test of refinement).
#include "pd_internal.h"
#include "pd_residual.h"

#include <cmath>

namespace {

constexpr int RB = 256;

__global__ void __launch_bounds__(RB)
residual_kernel(int n, int nbar, int ell, int dims, double tau, const double *__restrict__ u0,
                const double *__restrict__ F, const double *__restrict__ U,
                const double *__restrict__ coef, double *__restrict__ red) {
  __shared__ double sr[RB / 64], sg[RB / 64], su[RB / 64];
  double rn = 0.0, gn = 0.0, un = 0.0;
  // grid-stride walk over (t, i) with the stride split once into rows and
  // columns (no division per point)
  const size_t g0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t G = (size_t)gridDim.x * blockDim.x;
  const int dt = (int)(G / nbar), di = (int)(G % nbar);
  int t = (int)(g0 / nbar), i = (int)(g0 % nbar);
  while (t < ell) {
    double r, g;
    residual_point(t, i, n, nbar, dims, tau, u0, F, U, coef, r, g);
    // (M U)_{t,i}: Algorithm 3's test measures the residual against ||M U||_F
    const double *Ut = U + (size_t)t * nbar;
    double u = Ut[i];
    if (dims == 1) {
      u = coef[n + i] * Ut[i];
      if (i > 0) u += coef[i] * Ut[i - 1];
      if (i < n - 1) u += coef[2 * n + i] * Ut[i + 1];
    }
    rn += r * r;
    gn += g * g;
    un += u * u;
    t += dt;
    i += di;
    if (i >= nbar) { i -= nbar; ++t; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    rn += __shfl_down(rn, off, 64);
    gn += __shfl_down(gn, off, 64);
    un += __shfl_down(un, off, 64);
  }
  const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) { sr[wid] = rn; sg[wid] = gn; su[wid] = un; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int w = 0; w < RB / 64; ++w) { a += sr[w]; b += sg[w]; c += su[w]; }
    red[3 * blockIdx.x] = a;
    red[3 * blockIdx.x + 1] = b;
    red[3 * blockIdx.x + 2] = c;
  }
}

}  // namespace

// Up to 8192 blocks: each thread's points are a chain of dependent loads, so
// the pass needs many waves in flight to cover HBM latency (with 1024 blocks
// it ran at under 1 TB/s on the 8191 x 2048 workload).
int pd_residual_blocks(pd_plan p) {
  size_t total = (size_t)p->ell * p->nbar;
  size_t b = (total + RB - 1) / RB;
  return (int)(b < 8192 ? b : 8192);
}

// Sum the 2*nblk partial norms left in p->red by a residual pass.
pd_status pd_sum_norms(pd_plan p, int nblk, double *rn2, double *gn2) {
  std::vector<double> h(2 * (size_t)nblk);
  PD_HIP_CHECK(hipMemcpyAsync(h.data(), p->red, h.size() * sizeof(double),
                              hipMemcpyDeviceToHost, p->stream));
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nblk; ++i) { a += h[2 * i]; b += h[2 * i + 1]; }
  *rn2 = a;
  *gn2 = b;
  return PD_OK;
}

pd_status pd_residual_norms(pd_plan p, const double *u0, const double *F, const double *U,
                            double *rn2, double *gn2, double *un2) {
  const int nb = pd_residual_blocks(p);
  hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(RB), 0, p->stream, p->n, p->nbar, p->ell,
                     p->dims, p->tau, u0, F, U, p->coef64, p->red);
  PD_HIP_CHECK(hipGetLastError());
  std::vector<double> h(3 * (size_t)nb);
  PD_HIP_CHECK(hipMemcpyAsync(h.data(), p->red, h.size() * sizeof(double),
                              hipMemcpyDeviceToHost, p->stream));
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = 0; i < nb; ++i) { a += h[3 * i]; b += h[3 * i + 1]; c += h[3 * i + 2]; }
  if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c)) {
    pd_set_error("non-finite residual norm");
    return PD_ENONFINITE;
  }
  *rn2 = a;
  *gn2 = b;
  *un2 = c;
  return PD_OK;
}

pd_status pd_residual_impl(pd_plan p, const double *u0, const double *F, const double *U,
                           double *rel) {
  double a, b, c;
  pd_status st = pd_residual_norms(p, u0, F, U, &a, &b, &c);
  if (st != PD_OK) return st;
  *rel = (b > 0.0) ? std::sqrt(a / b) : std::sqrt(a);
  return PD_OK;
}
