// Standalone float64 residual of the all-at-once system,
// ||G - A(U)||_F / ||G||_F (Algorithm 3, the residual test on U_1; here the
// accuracy report of a solve and the stopping test of refinement).
#include "pd_internal.h"
#include "pd_residual.h"

#include <cmath>
#include <mutex>

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

// ---------------------------------------------------------------------------
// The allocation-free residual (paradiag_residual_noalloc): the per-block
// partial norms and their totals live in a file-scope device array instead
// of the plan's reduction buffer, and the totals are summed on the device, so
// the call allocates nothing on the device or the host.  Every call on a GPU
// shares that GPU's copy of the array; calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr int PD_NOALLOC_MAX_BLOCKS = 8192;
constexpr size_t PD_NOALLOC_SCRATCH_DOUBLES = 3 * (size_t)PD_NOALLOC_MAX_BLOCKS + 4;
static __device__ __align__(256) double scratch[PD_NOALLOC_SCRATCH_DOUBLES];

namespace {

std::mutex g_scratch_mu;
constexpr int PD_MAX_DEVICES = 64;
double *g_scratch_ptr[PD_MAX_DEVICES] = {};

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current (in host code the array's name is not a device
// address).
pd_status scratch_address(int device, double **out) {
  if (device < 0 || device >= PD_MAX_DEVICES) {
    pd_set_error("device index out of range for the scratch table");
    return PD_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    PD_HIP_CHECK(hipGetDevice(&cur));
    if (cur != device) PD_HIP_CHECK(hipSetDevice(device));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      pd_set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return PD_EHIP;
    }
    g_scratch_ptr[device] = static_cast<double *>(ptr);
  }
  *out = g_scratch_ptr[device];
  return PD_OK;
}

// Sum the 3 * nb partial norms in a fixed order (each thread a strided run,
// then a fixed tree in LDS) into tot[0..2].
__global__ void __launch_bounds__(RB) sum_partials_kernel(int nb, const double *__restrict__ red,
                                                          double *__restrict__ tot) {
  __shared__ double s[3][RB];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nb; i += RB) {
    a += red[3 * i];
    b += red[3 * i + 1];
    c += red[3 * i + 2];
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  s[2][threadIdx.x] = c;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 3; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) tot[threadIdx.x] = s[threadIdx.x][0];
}

}  // namespace

extern "C" pd_status paradiag_residual_noalloc(pd_plan p, const double *u0, const double *F,
                                               const double *U, double *rel) {
  if (!p || !rel || !u0 || !F || !U) {
    pd_set_error("invalid residual arguments");
    return PD_EINVAL;
  }
  if (p->bdf_s > 1) {
    pd_set_error("paradiag_residual_noalloc: backward-Euler plans only (bdf_order 1)");
    return PD_ENOTSUP;
  }
  const int nb = pd_residual_blocks(p);
  if (nb > PD_NOALLOC_MAX_BLOCKS || 3 * (size_t)nb + 3 > PD_NOALLOC_SCRATCH_DOUBLES) {
    pd_set_error("paradiag_residual_noalloc: the residual pass needs " + std::to_string(nb) +
                 " partial-norm blocks, above the static scratch's " +
                 std::to_string(PD_NOALLOC_MAX_BLOCKS));
    return PD_ENOTSUP;
  }
  double *sp = nullptr;
  pd_status st = scratch_address(p->device, &sp);
  if (st != PD_OK) return st;
  double *red = sp, *tot = sp + 3 * (size_t)PD_NOALLOC_MAX_BLOCKS;
  // every block writes its three partial norms, so nothing needs clearing
  hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(RB), 0, p->stream, p->n, p->nbar, p->ell,
                     p->dims, p->tau, u0, F, U, p->coef64, red);
  PD_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(RB), 0, p->stream, nb, red, tot);
  PD_HIP_CHECK(hipGetLastError());
  double h[3];
  PD_HIP_CHECK(hipMemcpyAsync(h, tot, sizeof(h), hipMemcpyDeviceToHost, p->stream));
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) {
    pd_set_error("non-finite residual norm");
    return PD_ENONFINITE;
  }
  *rel = (h[1] > 0.0) ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
  return PD_OK;
}

pd_status pd_residual_impl(pd_plan p, const double *u0, const double *F, const double *U,
                           double *rel, double *est) {
  double a, b, c;
  pd_status st = pd_residual_norms(p, u0, F, U, &a, &b, &c);
  if (st != PD_OK) return st;
  *rel = (b > 0.0) ? std::sqrt(a / b) : std::sqrt(a);
  if (est) *est = (p->err_factor > 0.0 && c > 0.0) ? p->err_factor * std::sqrt(a / c) : -1.0;
  return PD_OK;
}
