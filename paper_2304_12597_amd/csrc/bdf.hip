// BDF of order s in 2..6 (Section 5) on the stages of Algorithm 1.
//
// The all-at-once system (M + tau beta K) U - M U Sigma_s^T = G has
// Sigma_s = C_s - [e_1..e_s] A_s [e_{ell-s+1}..e_ell]^T: a circulant C_s
// (alpha_1..alpha_s below the diagonal, wrapped around) minus a rank-s
// term, A_s the s x s upper-triangular block of the wrapped entries,
// (A_s)_{k,c} = alpha_{s-c+k} for c >= k (0-based).  BDF plans carry the
// shifts lambda_i = 1 - pi_i, pi = F C_s e_1, and tau beta K in place of
// tau K, so the forward transform, the parfor of shifted solves with x = 0
// and the inverse transform of a real [ell][nbar] array X compute
//
//     Y(X) = IFFT(P^{-1} M FFT(X)),   P_i = (1 - pi_i) M + tau beta K.
//
// The pieces of the rank-s Sherman-Morrison-Woodbury solve are then
//   U_1 = Y(h) (G = M h),
//   b^(s)_k = sum_i gamma_i^(k) (P_i^{-1} Ghat)_i = sum_c (A_s)_{k,c} U_1[ell-s+c]:
//     gamma^(k) = F^{-T}[e_{ell-s+1}..e_ell] A_s^T e_k, so the weighted sum over
//     frequencies is the inverse transform sampled at the last s time rows;
//   (J^(s) v)_k = v_k + sum_c (A_s)_{k,c} Y(X(v))[ell-s+c]:
//     theta^(h) = F e_h, so sum_h theta_i^(h) v_h is the transform of X(v),
//     the array holding v_h in time row h-1 and zeros elsewhere;
//   U = U_1 - Y(X(x)) with x the solution of J^(s) x = b^(s).
// X(v) has s nonzero rows, so its transform is an s-term sum per frequency
// (bdf_spec_kernel), and only s rows of the inverse transform are needed:
// sum_c (A_s)_{k,c} Z[ell-s+c] = sum_i gamma_i^(k) Zhat_i, one weighted sum
// over the half spectrum per block (bdf_gather_kernel, weights 2 Re(.) for
// the conjugate halves).  A capacitance product is then one parfor of
// shifted solves between two streaming passes; #PinT = GMRES iterations + 2
// as for s = 1 (the block Galerkin method of bgal.hip: residual checks + 2).
#include "pd_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace {

constexpr int BB = 256;            // threads per block of the BDF kernels
constexpr int RES_ROWS = 64;       // time-row groups of the residual kernel

struct BdfAlpha {
  double a[6];                     // alpha_1..alpha_s
};
struct BdfBlock {
  double A[36];                    // A_s, row-major s x s
};

// out[t][i] = tau beta F[t][i] + sum_{j=t+1}^{s} alpha_j u_{t+1-j}[i]; u0s
// row r holds u_{r+1-s}.  Grid: (ceil(n/BB), ell).
__global__ void __launch_bounds__(BB)
bdf_rhs_kernel(int n, int s, double tb, BdfAlpha c, const double *__restrict__ u0s,
               const double *__restrict__ F, double *__restrict__ out) {
  const int i = blockIdx.x * BB + threadIdx.x;
  const int t = blockIdx.y;
  if (i >= n) return;
  const size_t idx = (size_t)t * n + i;
  double v = tb * F[idx];
  if (t < s)
    for (int j = t + 1; j <= s; ++j) v += c.a[j - 1] * u0s[(size_t)(s + t - j) * n + i];
  out[idx] = v;
}

// spec[f][i] = sign * sum_{h<s} v_h[i] exp(-2 pi i f h / ell), f = 0..ell/2:
// the half spectrum of X(v).  tw[m] = exp(-2 pi i m / ell), ell a power of
// two.  Grid: (ceil(n/BB), F2).
__global__ void __launch_bounds__(BB)
bdf_spec_kernel(int n, int ell, int s, double sign, const double *__restrict__ v,
                const cpx<double> *__restrict__ tw, cpx<double> *__restrict__ spec) {
  const int i = blockIdx.x * BB + threadIdx.x;
  const int f = blockIdx.y;
  if (i >= n) return;
  double re = 0.0, im = 0.0;
#pragma unroll
  for (int h = 0; h < 6; ++h)
    if (h < s) {
      const cpx<double> w = tw[(f * h) & (ell - 1)];
      const double x = sign * v[(size_t)h * n + i];
      re += w.re * x;
      im += w.im * x;
    }
  spec[(size_t)f * n + i] = cpx<double>{re, im};
}

// part[ch][k][i] = sum over the ch-th chunk of frequencies f of
// Re(g[k][f] Y[f][i]) (g = weight_f gamma_f^(k)).  Block: 64 columns x 4
// frequency lanes (a wave reads 64 consecutive entries of one frequency).
// Grid: (ceil(n/64), PD_BDF_GCH).
__global__ void __launch_bounds__(256)
bdf_gather_kernel(int n, int F2, int s, const cpx<double> *__restrict__ g,
                  const cpx<double> *__restrict__ Y, double *__restrict__ part) {
  __shared__ double sh[4][6][64];
  const int col = threadIdx.x & 63, lane = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + col;
  const int ch = blockIdx.y;
  const int per = (F2 + PD_BDF_GCH - 1) / PD_BDF_GCH;
  const int f0 = ch * per, f1 = (f0 + per < F2) ? f0 + per : F2;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < n)
    for (int f = f0 + lane; f < f1; f += 4) {
      const cpx<double> y = Y[(size_t)f * n + i];
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (k < s) {
          const cpx<double> w = g[(size_t)k * F2 + f];
          acc[k] += w.re * y.re - w.im * y.im;
        }
    }
#pragma unroll
  for (int k = 0; k < 6; ++k) sh[lane][k][col] = acc[k];
  __syncthreads();
  if (lane == 0 && i < n)
    for (int k = 0; k < s; ++k)
      part[((size_t)ch * s + k) * n + i] = sh[0][k][col] + sh[1][k][col] + sh[2][k][col] +
                                           sh[3][k][col];
}

// out[k][i] = v[k][i] (0 if v is NULL) + sum_ch part[ch][k][i] (fixed order).
// Grid: (ceil(n/BB), s).
__global__ void __launch_bounds__(BB)
bdf_finish_kernel(int n, int s, const double *__restrict__ v, const double *__restrict__ part,
                  double *__restrict__ out) {
  const int i = blockIdx.x * BB + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n) return;
  double acc = v ? v[(size_t)k * n + i] : 0.0;
  for (int ch = 0; ch < PD_BDF_GCH; ++ch) acc += part[((size_t)ch * s + k) * n + i];
  out[(size_t)k * n + i] = acc;
}

// out[k][i] = v[k][i] (0 if v is NULL) + sum_{c>=k} (A_s)_{k,c} Z[ell-s+c][i].
// Grid: (ceil(n/BB), s).
__global__ void __launch_bounds__(BB)
bdf_extract_kernel(int n, int ell, int s, BdfBlock A, const double *__restrict__ v,
                   const double *__restrict__ Z, double *__restrict__ out) {
  const int i = blockIdx.x * BB + threadIdx.x;
  const int k = blockIdx.y;
  if (i >= n) return;
  double acc = v ? v[(size_t)k * n + i] : 0.0;
  for (int c = k; c < s; ++c) acc += A.A[k * s + c] * Z[(size_t)(ell - s + c) * n + i];
  out[(size_t)k * n + i] = acc;
}

// Partial sums of ||G - A(U)||^2 and ||G||^2 for eq. discrete_probBDF:
// row t, with u_{t-j} from U (t - j >= 0) or the starting values,
//   G_t   = M (sum_{j>t} alpha_j u_{t+1-j} + tau beta f_t)   (0-based rows),
//   A(U)_t = (M + tau beta K) u_t - M sum_{j<=t} alpha_j u_{t-j}.
// Grid: (ceil(n/BB), RES_ROWS) blocks, time rows strided by gridDim.y;
// red[2 b], red[2 b + 1] for block b = y * gridDim.x + x.
__global__ void __launch_bounds__(BB)
bdf_residual_kernel(int n, int ell, int s, double tb, BdfAlpha c, const double *__restrict__ u0s,
                    const double *__restrict__ F, const double *__restrict__ U,
                    const double *__restrict__ coef, double *__restrict__ red) {
  __shared__ double sr[BB / 64], sg[BB / 64];
  const int i = blockIdx.x * BB + threadIdx.x;
  double rn = 0.0, gn = 0.0;
  if (i < n) {
    const double ML = coef[i], MD = coef[n + i], MU = coef[2 * n + i];
    const double KL = coef[3 * n + i], KD = coef[4 * n + i], KU = coef[5 * n + i];
    for (int t = blockIdx.y; t < ell; t += gridDim.y) {
      // g(ii): G_t / M at column ii; w(ii): everything M multiplies in
      // G_t - A(U)_t, i.e. g + sum_{j<=t} alpha_j u_{t-j} - u_t
      auto gw = [&](int ii, double &g, double &w) {
        g = tb * F[(size_t)t * n + ii];
        w = -U[(size_t)t * n + ii];
        for (int j = 1; j <= s; ++j) {
          if (j > t) g += c.a[j - 1] * u0s[(size_t)(s + t - j) * n + ii];
          else w += c.a[j - 1] * U[(size_t)(t - j) * n + ii];
        }
        w += g;
      };
      double g0, w0;
      gw(i, g0, w0);
      double g = MD * g0, r = MD * w0 - KD * U[(size_t)t * n + i];
      if (i > 0) {
        double gl, wl;
        gw(i - 1, gl, wl);
        g += ML * gl;
        r += ML * wl - KL * U[(size_t)t * n + i - 1];
      }
      if (i < n - 1) {
        double gu, wu;
        gw(i + 1, gu, wu);
        g += MU * gu;
        r += MU * wu - KU * U[(size_t)t * n + i + 1];
      }
      rn += r * r;
      gn += g * g;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    rn += __shfl_down(rn, off, 64);
    gn += __shfl_down(gn, off, 64);
  }
  const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    sr[wid] = rn;
    sg[wid] = gn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < BB / 64; ++w) {
      a += sr[w];
      b += sg[w];
    }
    const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    red[2 * blk] = a;
    red[2 * blk + 1] = b;
  }
}

// 2D (M = I, K = I (x) T + T (x) I, coef holding tau beta T): partial sums of
// ||G - A(U)||^2 and ||G||^2 at the points i = y n + x of every time row t,
//   G_t = sum_{j>t} alpha_j u_{t+1-j} + tau beta f_t,
//   A(U)_t = u_t + tau beta K u_t - sum_{j<=t} alpha_j u_{t-j}.
// Grid: (ceil(nbar/BB), RES_ROWS); red as for the 1D kernel.
__global__ void __launch_bounds__(BB)
bdf_residual2d_kernel(int n, int ell, int s, double tb, BdfAlpha c,
                      const double *__restrict__ u0s, const double *__restrict__ F,
                      const double *__restrict__ U, const double *__restrict__ coef,
                      double *__restrict__ red) {
  __shared__ double sr[BB / 64], sg[BB / 64];
  const int nbar = n * n;
  const int i = blockIdx.x * BB + threadIdx.x;
  double rn = 0.0, gn = 0.0;
  if (i < nbar) {
    const int y = i / n, x = i - y * n;
    const double *KL = coef + 3 * n, *KD = coef + 4 * n, *KU = coef + 5 * n;
    for (int t = blockIdx.y; t < ell; t += gridDim.y) {
      const double *Ut = U + (size_t)t * nbar;
      double g = tb * F[(size_t)t * nbar + i];
      double w = -Ut[i];
      for (int j = 1; j <= s; ++j) {
        if (j > t) g += c.a[j - 1] * u0s[(size_t)(s + t - j) * nbar + i];
        else w += c.a[j - 1] * U[(size_t)(t - j) * nbar + i];
      }
      double ku = (KD[x] + KD[y]) * Ut[i];
      if (x > 0) ku += KL[x] * Ut[i - 1];
      if (x < n - 1) ku += KU[x] * Ut[i + 1];
      if (y > 0) ku += KL[y] * Ut[i - n];
      if (y < n - 1) ku += KU[y] * Ut[i + n];
      const double r = w + g - ku;
      rn += r * r;
      gn += g * g;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    rn += __shfl_down(rn, off, 64);
    gn += __shfl_down(gn, off, 64);
  }
  const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    sr[wid] = rn;
    sg[wid] = gn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < BB / 64; ++w) {
      a += sr[w];
      b += sg[w];
    }
    const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    red[2 * blk] = a;
    red[2 * blk + 1] = b;
  }
}

BdfAlpha alpha_of(pd_plan p) {
  BdfAlpha c;
  for (int j = 0; j < 6; ++j) c.a[j] = p->bdf_alpha[j];
  return c;
}

BdfBlock block_of(pd_plan p) {
  BdfBlock B;
  const int s = p->bdf_s;
  for (int q = 0; q < 36; ++q) B.A[q] = 0.0;
  for (int k = 0; k < s; ++k)
    for (int c = k; c < s; ++c) B.A[k * s + c] = p->bdf_alpha[s - c + k - 1];
  return B;
}

bool bdf_plan_ok(pd_plan p) {
  if (p->bdf_s < 2 || p->bdf_s > 6 || !p->wreal || !p->wz || !p->bdf_g ||
      p->ell < 2 * p->bdf_s || (p->dims == 2 && (!p->bdf_h || !p->bdf_t))) {
    pd_set_error("not a BDF plan of order > 1");
    return false;
  }
  return true;
}

// p->spec = the half spectrum of X(sign * v); 2D plans first take the s
// rows of v to the DST-x domain of the shifted solves.
pd_status spectrum_of(pd_plan p, const double *v, double sign) {
  const int n = p->nbar;
  if (p->dims == 2) {
    pd_status st = pd_launch_dst_x_rows(p, v, p->bdf_t, p->bdf_s, 0);
    if (st != PD_OK) return st;
    v = p->bdf_t;
  }
  hipLaunchKernelGGL(bdf_spec_kernel, dim3((n + BB - 1) / BB, p->F2), dim3(BB), 0, p->stream, n,
                     p->ell, p->bdf_s, sign, v, reinterpret_cast<const cpx<double> *>(p->tw64),
                     reinterpret_cast<cpx<double> *>(p->spec));
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// out (= or +=) the inverse transform of P^{-1} M FFT(p->wreal): forward
// transform, shifted solves with x = 0 in place, inverse transform (2D: p->wreal
// is in the DST-x domain and the result is taken back to space).
pd_status transform_solve(pd_plan p, double *out, int accumulate) {
  pd_status st = pd_launch_fft_forward(p, nullptr, p->wreal, nullptr, p->spec, 2);
  if (st != PD_OK) return st;
  st = pd_launch_tridiag(p, 1, p->spec, nullptr, p->spec);
  if (st != PD_OK) return st;
  return pd_inverse(p, p->spec, out, accumulate);
}

pd_status extract(pd_plan p, const double *v, const double *Z, double *out) {
  const int n = p->nbar, s = p->bdf_s;
  hipLaunchKernelGGL(bdf_extract_kernel, dim3((n + BB - 1) / BB, s), dim3(BB), 0, p->stream, n,
                     p->ell, s, block_of(p), v, Z, out);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

}  // namespace

int pd_bdf_residual_blocks(pd_plan p) {
  return ((p->nbar + BB - 1) / BB) * std::min(p->ell, RES_ROWS);
}

pd_status pd_bdf_rhs(pd_plan p, const double *u0s, const double *F, double *out) {
  if (!bdf_plan_ok(p)) return PD_ENOTSUP;
  const int n = p->nbar;
  hipLaunchKernelGGL(bdf_rhs_kernel, dim3((n + BB - 1) / BB, p->ell), dim3(BB), 0, p->stream, n,
                     p->bdf_s, p->tau * p->bdf_beta, alpha_of(p), u0s, F, out);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_bdf_apply(pd_plan p, const double *v, double *Jv) {
  if (!bdf_plan_ok(p)) return PD_ENOTSUP;
  const int n = p->nbar, s = p->bdf_s;
  pd_status st = spectrum_of(p, v, 1.0);
  if (st != PD_OK) return st;
  st = pd_launch_tridiag(p, 1, p->spec, nullptr, p->spec);
  if (st != PD_OK) return st;
  hipLaunchKernelGGL(bdf_gather_kernel, dim3((n + 63) / 64, PD_BDF_GCH), dim3(256), 0, p->stream,
                     n, p->F2, s, reinterpret_cast<const cpx<double> *>(p->bdf_g),
                     reinterpret_cast<const cpx<double> *>(p->spec), p->wz);
  if (p->dims == 1) {
    hipLaunchKernelGGL(bdf_finish_kernel, dim3((n + BB - 1) / BB, s), dim3(BB), 0, p->stream, n,
                       s, v, p->wz, Jv);
    PD_HIP_CHECK(hipGetLastError());
    return PD_OK;
  }
  // 2D: the s rows come out in the DST-x domain: Jv = v + DST-x(rows)
  hipLaunchKernelGGL(bdf_finish_kernel, dim3((n + BB - 1) / BB, s), dim3(BB), 0, p->stream, n,
                     s, nullptr, p->wz, p->bdf_t);
  PD_HIP_CHECK(hipGetLastError());
  if (Jv != v)
    PD_HIP_CHECK(hipMemcpyAsync(Jv, v, sizeof(double) * (size_t)s * n, hipMemcpyDeviceToDevice,
                                p->stream));
  return pd_launch_dst_x_rows(p, p->bdf_t, Jv, s, 1);
}

pd_status pd_bdf_residual_norms(pd_plan p, const double *u0s, const double *F,
                                const double *U, double *rn2, double *gn2) {
  if (!bdf_plan_ok(p)) return PD_ENOTSUP;
  const int n = p->n;
  const int gy = std::min(p->ell, RES_ROWS);
  const int nb = pd_bdf_residual_blocks(p);
  if (p->dims == 1)
    hipLaunchKernelGGL(bdf_residual_kernel, dim3((n + BB - 1) / BB, gy), dim3(BB), 0, p->stream,
                       n, p->ell, p->bdf_s, p->tau * p->bdf_beta, alpha_of(p), u0s, F, U,
                       p->coef64, p->red);
  else
    hipLaunchKernelGGL(bdf_residual2d_kernel, dim3((p->nbar + BB - 1) / BB, gy), dim3(BB), 0,
                       p->stream, n, p->ell, p->bdf_s, p->tau * p->bdf_beta, alpha_of(p), u0s, F,
                       U, p->coef64, p->red);
  PD_HIP_CHECK(hipGetLastError());
  std::vector<double> h(2 * (size_t)nb);
  PD_HIP_CHECK(hipMemcpyAsync(h.data(), p->red, h.size() * sizeof(double),
                              hipMemcpyDeviceToHost, p->stream));
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nb; ++q) {
    a += h[2 * q];
    b += h[2 * q + 1];
  }
  if (!std::isfinite(a) || !std::isfinite(b)) {
    pd_set_error("non-finite residual norm");
    return PD_ENONFINITE;
  }
  *rn2 = a;
  *gn2 = b;
  return PD_OK;
}

// The whole BDF solve: h, U_1 = Y(h) into U, b^(s), J^(s) x = b^(s) by
// GMRES or by the block Galerkin method (krylov = PD_KRYLOV_FOM),
// U -= Y(X(x)) (the transform of X(x) as an s-term sum).
pd_status pd_bdf_solve(pd_plan p, const double *u0s, const double *F, double *U, double tol,
                       pd_info *info) {
  if (!bdf_plan_ok(p)) return PD_ENOTSUP;
  // h into the transform input (2D: into bdf_h, then to the DST-x domain)
  pd_status st = pd_bdf_rhs(p, u0s, F, p->dims == 2 ? p->bdf_h : p->wreal);
  if (st != PD_OK) return st;
  if (p->dims == 2) {
    st = pd_launch_dst_x_rows(p, p->bdf_h, p->wreal, p->ell, 0);
    if (st != PD_OK) return st;
  }
  st = transform_solve(p, U, 0);
  if (st != PD_OK) return st;
  st = extract(p, nullptr, U, p->bvec);
  if (st != PD_OK) return st;
  int its = 0, checks = 0;
  double rr = 0.0;
  pd_status gst;
  if (p->krylov == PD_KRYLOV_FOM && p->dims == 2) {
    // the block Galerkin method works in the DST-x domain of the line solves:
    // b^(s) there (its s rows), x back to space
    const size_t sn = (size_t)p->bdf_s * p->nbar;
    double *bd = p->wz, *xd = p->wz + sn;
    st = pd_launch_dst_x_rows(p, p->bvec, bd, p->bdf_s, 0);
    if (st != PD_OK) return st;
    gst = pd_bgal(p, bd, xd, tol * PD_GMRES_TOL_FACTOR, &its, &rr, &checks);
    if (gst != PD_OK && gst != PD_ENOTCONV) return gst;
    st = pd_launch_dst_x_rows(p, xd, p->xvec, p->bdf_s, 0);
    if (st != PD_OK) return st;
  } else {
    gst = p->krylov == PD_KRYLOV_FOM
              ? pd_bgal(p, p->bvec, p->xvec, tol * PD_GMRES_TOL_FACTOR, &its, &rr, &checks)
              : pd_gmres(p, p->bvec, p->xvec, tol * PD_GMRES_TOL_FACTOR, &its, &rr);
    if (gst != PD_OK && gst != PD_ENOTCONV) return gst;
  }
  st = spectrum_of(p, p->xvec, -1.0);
  if (st != PD_OK) return st;
  st = pd_launch_tridiag(p, 1, p->spec, nullptr, p->spec);
  if (st != PD_OK) return st;
  st = pd_inverse(p, p->spec, U, 1);
  if (st != PD_OK) return st;
  if (info) {
    info->gmres_iters = its;
    info->pint_loops = (p->krylov == PD_KRYLOV_FOM ? checks : its) + 2;
    info->sweeps = 1;
    info->gmres_rel_residual = rr;
  }
  if (p->check_residual) {
    double rn2, gn2;
    st = pd_bdf_residual_norms(p, u0s, F, U, &rn2, &gn2);
    if (st != PD_OK) return st;
    if (info) info->rel_residual = gn2 > 0.0 ? std::sqrt(rn2 / gn2) : std::sqrt(rn2);
  }
  PD_HIP_CHECK(hipStreamSynchronize(p->stream));
  if (gst == PD_ENOTCONV) pd_set_error("tolerance not reached");
  return gst;
}
