// Algorithm 2: the FOM-like projection of the capacitance system
// J_ell x = b onto a polynomial Krylov space, on the GPU.
//
// With the mass matrix the operator is A = tau M^{-1} K, so that every
// shifted block is P_i^{-1} M = (lambda_i I + A)^{-1} (lambda_i = 1 - pi_i)
// and K_m(A, b) is the paper's K_m(K, b) when M = I.  From the Arnoldi
// relation A V_m = V_m T_m + t v_{m+1} e_m^T (t = t_{m+1,m}):
//   S_i = (lambda_i I_m + T_m)^{-1},  h_i = P_i^{-1} M v_{m+1},
//   (I + w sum_i gamma_i (I - t V_m^T h_i e_m^T) S_i) y = beta e_1,
//   ||r|| = |t| w || (I - V_m V_m^T) sum_i gamma_i h_i e_m^T S_i y ||
// (Section 3, eq. compute_ym and eq. compute_resnorm; w = alpha^(1/ell),
// Section 4).  The sums over the full spectrum use its conjugate halves
// (real data: twice the real part for k = 1..ell/2-1).
//
// One Krylov step: u = tau K v (stencil) and w = M^{-1} u (one block, the
// partition solve), then two classical Gram-Schmidt passes.  Every q-th step
// (and at the cap) the residual check: all h_i at once through the pass-C
// shifted-solve kernel on a zero spectrum (one parfor: it writes -w h_i),
// V_m^T h_i, per frequency S_i by Gauss-Jordan, the m x m system for y, the
// weighted sum z = sum_i c_i h_i and the projected norm.
#include "pd_internal.h"
#include "pd_gj.h"
#include "pd_partition.h"
#include "pd_proj.h"

#include <cmath>
#include <vector>

namespace {

constexpr int FB = 512;    // single-block kernels
constexpr int FR = 16;     // rows per thread of the single-block kernels (n <= FB*FR)

// Sum over the block, returned to every thread, in a fixed order.
__device__ double block_sum(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
  return s;
}

// beta = ||b||, v_1 = b / beta, T = 0, state[0] = beta
__global__ void __launch_bounds__(FB)
fom_start_kernel(int n, const double *__restrict__ b, double *__restrict__ V,
                 double *__restrict__ T, int tsize, double *__restrict__ state) {
  __shared__ double red[FB / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += FB) s += b[i] * b[i];
  const double beta = sqrt(block_sum(s, red));
  for (int i = threadIdx.x; i < n; i += FB) V[i] = beta > 0.0 ? b[i] / beta : 0.0;
  for (int i = threadIdx.x; i < tsize; i += FB) T[i] = 0.0;
  if (threadIdx.x == 0) state[0] = beta;
}

// w = M^{-1} (tau K) v: stencil, then the partition solve with the uniform
// mass factors (16 rows per thread, P = ceil(n/16) threads).
__global__ void __launch_bounds__(512)
fom_apply_kernel(int n, const double *__restrict__ v, const cpx<double> *__restrict__ mfac,
                 double ml, double mu, double kl, double kd, double ku,
                 double *__restrict__ w) {
  constexpr int MR = 16;
  __shared__ cpx<double> lfac[6 * (MR - 1)];
  __shared__ Row3<double> xch[512];
  const int P = blockDim.x, lt = threadIdx.x;
  for (int i = lt; i < 6 * (MR - 1); i += P) lfac[i] = mfac[i];
  const int s0 = lt * MR;
  int len = n - s0;
  len = len < 0 ? 0 : (len > MR ? MR : len);
  cpx<double> d[MR];
#pragma unroll
  for (int q = 0; q < MR; ++q) {
    const int i = s0 + q;
    double u = 0.0;
    if (q < len) {
      u = kd * v[i];
      if (i > 0) u += kl * v[i - 1];
      if (i < n - 1) u += ku * v[i + 1];
    }
    d[q] = cpx<double>{u, 0.0};
  }
  __syncthreads();   // lfac visible
  partition_solve<double, MR>(d, len, lt, P, lfac, xch, cpx<double>{ml, 0.0},
                              cpx<double>{mu, 0.0});
#pragma unroll
  for (int q = 0; q < MR; ++q)
    if (q < len) w[s0 + q] = d[q].re;
}

// Two classical Gram-Schmidt passes of w against v_1..v_m (V rows 0..m-1),
// T[k][m-1] (row-major, FM_ columns), t = ||w||, V row m = w / t.
template <int FM_>
__global__ void __launch_bounds__(FB)
fom_orth_kernel(int n, int m, double *__restrict__ V, const double *__restrict__ wsrc,
                double *__restrict__ T) {
  __shared__ double red[FB / 64];
  __shared__ double part[FM_][FB / 64];
  __shared__ double dots[FM_];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63, nw = FB / 64;
  double wv[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int i = tid + r * FB;
    wv[r] = i < n ? wsrc[i] : 0.0;
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int k = 0; k < m; ++k) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < FR; ++r) {
        const int i = tid + r * FB;
        if (i < n) s += V[(size_t)k * n + i] * wv[r];
      }
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) part[k][wid] = s;
    }
    __syncthreads();
    if (tid < m) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += part[tid][q];
      dots[tid] = s;
      T[(size_t)tid * FM_ + (m - 1)] += s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const int i = tid + r * FB;
      if (i < n)
        for (int k = 0; k < m; ++k) wv[r] -= dots[k] * V[(size_t)k * n + i];
    }
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < FR; ++r) s += wv[r] * wv[r];
  const double t = sqrt(block_sum(s, red));
  if (tid == 0) T[(size_t)m * FM_ + (m - 1)] = t;
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int i = tid + r * FB;
    if (i < n) V[(size_t)m * n + i] = t > 0.0 ? wv[r] / t : 0.0;
  }
}

// proj[i][k] = s * sum_rows V[k][row] * hs_i[row] (hs holds -w h_i;
// s = -1/w).  Grid: (ceil(F2 / PROJ_PT), ceil(m / PROJ_PK)) tiles.
template <int FM_>
__global__ void __launch_bounds__(256)
fom_proj_kernel(int n, int F2, int m, const cpx<double> *__restrict__ hs,
                const double *__restrict__ V, double s, cpx<double> *__restrict__ proj) {
  const int i0 = blockIdx.x * PROJ_PT, k0 = blockIdx.y * PROJ_PK;
  cpx<double> v;
  proj_tile(n, F2, m, V, hs, i0, k0, v);
  const int t = threadIdx.x;
  if (t < PROJ_PK * PROJ_PT) {
    const int k = k0 + t / PROJ_PT, i = i0 + t % PROJ_PT;
    if (k < m && i < F2) proj[(size_t)i * FM_ + k] = cpx<double>{s * v.re, s * v.im};
  }
}

// Per frequency i (one wave each): S_i = (lambda_i I + T_m)^{-1} by
// Gauss-Jordan in LDS (wave_gj_inverse); the last row of S_i, and
// Zpart_i = Re(w g_i (S_i - t p_i (e_m^T S_i))) (g_i = weight * gamma_i, the
// conjugate half folded in).  Lane c writes column c.
template <int FM_>
__global__ void __launch_bounds__(64)
fom_small_kernel(int F2, int m, const double *__restrict__ lam, const double *__restrict__ gB,
                 double w, const double *__restrict__ T, const cpx<double> *__restrict__ proj,
                 double *__restrict__ Zpart, cpx<double> *__restrict__ lastrow) {
  using Cx = cpx<double>;
  __shared__ Cx a[FM_][2 * FM_];
  __shared__ Cx fcol[FM_];
  const int i = blockIdx.x, c = threadIdx.x;
  wave_gj_inverse<FM_>(m, Cx{lam[2 * i], lam[2 * i + 1]}, T, FM_, a, fcol);
  // S_i = right half of a
  if (c >= m) return;
  const double t = T[(size_t)m * FM_ + (m - 1)];
  const Cx g = {w * gB[2 * i], w * gB[2 * i + 1]};
  const Cx last = a[m - 1][m + c];
  lastrow[(size_t)i * FM_ + c] = last;
  for (int r = 0; r < m; ++r) {
    const Cx pr = proj[(size_t)i * FM_ + r];
    const Cx e = csub(a[r][m + c], cmul(Cx{t * pr.re, t * pr.im}, last));
    Zpart[(size_t)i * FM_ * FM_ + r * FM_ + c] = g.re * e.re - g.im * e.im;
  }
}

constexpr int ZCH = 16;   // frequency chunks of the Galerkin-matrix sums

// zp[ch][r][c] = sum over the ch-th chunk of frequencies of Zpart_i[r][c].
// Grid: (ceil(m^2 / 256), ZCH).
template <int FM_>
__global__ void __launch_bounds__(256)
fom_zsum_kernel(int F2, int m, const double *__restrict__ Zpart, double *__restrict__ zp) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int ch = blockIdx.y;
  if (e >= m * m) return;
  const int r = e / m, c = e - r * m;
  const int per = (F2 + ZCH - 1) / ZCH;
  const int i0 = ch * per, i1 = (i0 + per < F2) ? i0 + per : F2;
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += Zpart[(size_t)i * FM_ * FM_ + r * FM_ + c];
  zp[(size_t)ch * FM_ * FM_ + r * FM_ + c] = s;
}

// Z = I + sum of the chunk sums (fixed order), y = Z^{-1} beta e_1 (partial
// pivoting), c_i = g_i (e_m^T S_i y).
template <int FM_>
__global__ void __launch_bounds__(FB)
fom_solve_kernel(int F2, int m, const double *__restrict__ zp,
                 const cpx<double> *__restrict__ lastrow, const double *__restrict__ gB,
                 const double *__restrict__ state, double *__restrict__ y,
                 cpx<double> *__restrict__ cvec) {
  __shared__ double Z[FM_][FM_ + 1];
  __shared__ double ys[FM_];
  const int tid = threadIdx.x;
  for (int e = tid; e < m * m; e += FB) {
    const int r = e / m, c = e - r * m;
    double s = (r == c) ? 1.0 : 0.0;
    for (int ch = 0; ch < ZCH; ++ch) s += zp[(size_t)ch * FM_ * FM_ + r * FM_ + c];
    Z[r][c] = s;
  }
  for (int r = tid; r < m; r += FB) Z[r][FM_] = (r == 0) ? state[0] : 0.0;
  __syncthreads();
  // Gaussian elimination with partial pivoting, the rows below the pivot
  // updated in parallel
  for (int col = 0; col < m; ++col) {
    if (tid == 0) {
      int piv = col;
      for (int r = col + 1; r < m; ++r)
        if (fabs(Z[r][col]) > fabs(Z[piv][col])) piv = r;
      if (piv != col)
        for (int c = 0; c <= FM_; ++c) {
          const double t = Z[col][c];
          Z[col][c] = Z[piv][c];
          Z[piv][c] = t;
        }
    }
    __syncthreads();
    const int r = col + 1 + tid;
    if (r < m) {
      const double f = Z[r][col] / Z[col][col];
      for (int c = col; c < m; ++c) Z[r][c] -= f * Z[col][c];
      Z[r][FM_] -= f * Z[col][FM_];
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int r = m - 1; r >= 0; --r) {
      double s = Z[r][FM_];
      for (int c = r + 1; c < m; ++c) s -= Z[r][c] * ys[c];
      ys[r] = s / Z[r][r];
    }
    for (int r = 0; r < m; ++r) y[r] = ys[r];
  }
  __syncthreads();
  for (int i = tid; i < F2; i += FB) {
    cpx<double> s = {0.0, 0.0};
    for (int c = 0; c < m; ++c) {
      const cpx<double> l = lastrow[(size_t)i * FM_ + c];
      s.re += l.re * ys[c];
      s.im += l.im * ys[c];
    }
    const cpx<double> g = {gB[2 * i], gB[2 * i + 1]};
    cvec[i] = cmul(g, s);
  }
}

constexpr int WCH = 16;   // frequency chunks of the weighted sum

// zpart[ch][row] = sum over the ch-th chunk of frequencies of Re(c_i hs_i[row]).
// Block: 64 rows x 4 frequency lanes; grid (ceil(n/64), WCH).
__global__ void __launch_bounds__(256)
fom_wsum_kernel(int n, int F2, const cpx<double> *__restrict__ hs,
                const cpx<double> *__restrict__ cvec, double *__restrict__ zpart) {
  __shared__ double sh[4][64];
  const int col = threadIdx.x & 63, lane = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + col, ch = blockIdx.y;
  const int per = (F2 + WCH - 1) / WCH;
  const int i0 = ch * per, i1 = (i0 + per < F2) ? i0 + per : F2;
  double acc = 0.0;
  if (row < n)
    for (int i = i0 + lane; i < i1; i += 4) {
      const cpx<double> h = hs[(size_t)i * n + row], c = cvec[i];
      acc += c.re * h.re - c.im * h.im;
    }
  sh[lane][col] = acc;
  __syncthreads();
  if (lane == 0 && row < n)
    zpart[(size_t)ch * n + row] = sh[0][col] + sh[1][col] + sh[2][col] + sh[3][col];
}

// z[row] = s * sum_ch zpart[ch][row] (hs = -w h, s = -1/w)
__global__ void __launch_bounds__(256)
fom_wfinish_kernel(int n, const double *__restrict__ zpart, double s, double *__restrict__ z) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double acc = 0.0;
  for (int ch = 0; ch < WCH; ++ch) acc += zpart[(size_t)ch * n + row];
  z[row] = s * acc;
}

// rho = (I - V_m V_m^T) z (two passes), state[1] = |t| w ||rho||
template <int FM_>
__global__ void __launch_bounds__(FB)
fom_resid_kernel(int n, int m, const double *__restrict__ V, const double *__restrict__ z,
                 const double *__restrict__ T, double w, double *__restrict__ state) {
  __shared__ double red[FB / 64];
  __shared__ double part[FM_][FB / 64];
  __shared__ double dots[FM_];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63, nw = FB / 64;
  double zv[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int i = tid + r * FB;
    zv[r] = i < n ? z[i] : 0.0;
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int k = 0; k < m; ++k) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < FR; ++r) {
        const int i = tid + r * FB;
        if (i < n) s += V[(size_t)k * n + i] * zv[r];
      }
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) part[k][wid] = s;
    }
    __syncthreads();
    if (tid < m) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += part[tid][q];
      dots[tid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const int i = tid + r * FB;
      if (i < n)
        for (int k = 0; k < m; ++k) zv[r] -= dots[k] * V[(size_t)k * n + i];
    }
    __syncthreads();
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < FR; ++r) s += zv[r] * zv[r];
  const double nrm = sqrt(block_sum(s, red));
  if (tid == 0) state[1] = fabs(T[(size_t)m * FM_ + (m - 1)]) * w * nrm;
}

// Multi-block vector kernels (2D plans, n up to 1023^2): classical
// Gram-Schmidt and norms with per-block partial sums reduced by every block
// in a fixed order.
constexpr int MB = 256;
constexpr int MB_MAX_BLOCKS = 256;
constexpr int MCAP = 40;   // basis vectors a multi-block orthogonalisation handles

int fom_vec_blocks(int n) {
  const int b = (n + MB - 1) / MB;
  return b < MB_MAX_BLOCKS ? b : MB_MAX_BLOCKS;
}

// part[b * (cnt + 1) + k] = block b's share of V_k . w (k < cnt) and of
// w . w (k = cnt).
__global__ void __launch_bounds__(MB)
fom_mdots_kernel(int n, int cnt, const double *__restrict__ V, const double *__restrict__ w,
                 double *__restrict__ part) {
  __shared__ double red[MB / 64];
  for (int k = 0; k <= cnt; ++k) {
    double acc = 0.0;
    for (int row = blockIdx.x * MB + threadIdx.x; row < n; row += gridDim.x * MB) {
      const double wr = w[row];
      acc += (k < cnt ? V[(size_t)k * n + row] : wr) * wr;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * (cnt + 1) + k] = acc;
  }
}

// d_k = sum_b part[b][k]; w -= sum_k d_k V_k on the block's rows; block 0
// adds d_k to T[k * ldT + col] (T may be NULL).
__global__ void __launch_bounds__(MB)
fom_mupdate_kernel(int n, int cnt, int nblk, const double *__restrict__ part,
                   const double *__restrict__ V, double *__restrict__ w, double *__restrict__ T,
                   int ldT, int col) {
  __shared__ double d[MCAP];
  for (int k = threadIdx.x; k < cnt; k += MB) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * (cnt + 1) + k];
    d[k] = acc;
    if (T && blockIdx.x == 0) T[(size_t)k * ldT + col] += acc;
  }
  __syncthreads();
  for (int row = blockIdx.x * MB + threadIdx.x; row < n; row += gridDim.x * MB) {
    double v = w[row];
    for (int k = 0; k < cnt; ++k) v -= d[k] * V[(size_t)k * n + row];
    w[row] = v;
  }
}

// t = sqrt(sum_b part[b]) with part from a w . w pass (fom_mdots_kernel with
// cnt = 0, one value per block); V row cnt = w / t (0 if t = 0); block 0
// writes t to T[cnt * ldT + col] (T != NULL) and to *tout (tout != NULL).
__global__ void __launch_bounds__(MB)
fom_mscale_kernel(int n, int cnt, int nblk, const double *__restrict__ part,
                  const double *__restrict__ w, double *__restrict__ V, double *__restrict__ T,
                  int ldT, int col, double *__restrict__ tout) {
  __shared__ double tsh;
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += part[b];
    tsh = sqrt(acc);
    if (blockIdx.x == 0) {
      if (T) T[(size_t)cnt * ldT + col] = tsh;
      if (tout) *tout = tsh;
    }
  }
  __syncthreads();
  const double t = tsh;
  for (int row = blockIdx.x * MB + threadIdx.x; row < n; row += gridDim.x * MB)
    V[(size_t)cnt * n + row] = t > 0.0 ? w[row] / t : 0.0;
}

// out[0] = (acc ? out[0] : 0) + sum_b part[b][0]
__global__ void fom_maccum_kernel(int nblk, const double *__restrict__ part, int acc,
                                  double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = acc ? out[0] : 0.0;
  for (int b = 0; b < nblk; ++b) s += part[b];
  out[0] = s;
}

// state[1] = |t_{m+1,m}| w sqrt(sum_b part[b][0]) (the projected norm of z)
__global__ void fom_mres_kernel(int nblk, const double *__restrict__ part,
                                const double *__restrict__ T, int ldT, int m, double w,
                                double *__restrict__ state) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += part[b];
  state[1] = fabs(T[(size_t)m * ldT + (m - 1)]) * w * sqrt(acc);
}

// 2D plans, in the DST-x domain of the line solves (index y * n + j, x-mode
// j + 1): w = tau K v with tau K = diag(theta_j) along x plus tau T along y,
// theta_j = tkd + 2 tku cos(pi (j + 1) / (n + 1)) (cosx[j], from the plan).
__global__ void __launch_bounds__(256)
fom_apply2d_kernel(int n, const double *__restrict__ v, const double *__restrict__ cosx,
                   double tkl, double tkd, double tku, double *__restrict__ w) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * n) return;
  const int y = idx / n, j = idx - y * n;
  const double th = tkd + 2.0 * tku * cosx[j];
  double val = (th + tkd) * v[idx];
  if (y > 0) val += tkl * v[idx - n];
  if (y < n - 1) val += tku * v[idx + n];
  w[idx] = val;
}

// x = V_m y
__global__ void __launch_bounds__(256)
fom_combine_kernel(int n, int m, const double *__restrict__ V, const double *__restrict__ y,
                   double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < m; ++k) s += y[k] * V[(size_t)k * n + i];
  x[i] = s;
}

}  // namespace

// Host side --------------------------------------------------------------

size_t pd_fom_doubles(int n, int F2) {
  const size_t FM = PD_FOM_MAXM;
  return (FM + 1) * FM                // T
         + 2 * (size_t)F2 * FM        // proj
         + (size_t)F2 * FM * FM       // Zpart
         + 2 * (size_t)F2 * FM        // last rows of S_i
         + FM                         // y
         + 2 * (size_t)F2             // c_i
         + 4                          // beta, residual
         + 12 * 15                    // mass factors (16 rows per thread)
         + (size_t)n                  // z
         + (size_t)WCH * n            // chunk partials of z
         + (size_t)ZCH * FM * FM      // chunk sums of the Galerkin matrix
         + (size_t)MB_MAX_BLOCKS * MCAP;   // multi-block partial sums
}

bool pd_fom_supported(pd_plan p) {
  if (p->prec != PD_FP64 || !p->uniform) return false;
  return p->dims == 2 || p->n <= FB * FR;
}

size_t pd_fom_mfac_offset(int F2) {
  const size_t FM = PD_FOM_MAXM;
  return (FM + 1) * FM + 2 * (size_t)F2 * FM + (size_t)F2 * FM * FM + 2 * (size_t)F2 * FM + FM +
         2 * (size_t)F2 + 4;
}

pd_status pd_fom(pd_plan p, const double *b, double *x, double rtol, int *iters,
                 double *relres, int *checks) {
  constexpr int FM = PD_FOM_MAXM;
  const int n = p->nbar, F2 = p->F2;
  const int maxm = p->maxit < FM ? p->maxit : FM;
  const int q = p->fom_q < 1 ? 1 : p->fom_q;
  double *T = p->fom;
  auto proj = reinterpret_cast<cpx<double> *>(T + (FM + 1) * FM);
  double *Zpart = reinterpret_cast<double *>(proj + (size_t)F2 * FM);
  auto lastrow = reinterpret_cast<cpx<double> *>(Zpart + (size_t)F2 * FM * FM);
  double *y = reinterpret_cast<double *>(lastrow + (size_t)F2 * FM);
  auto cvec = reinterpret_cast<cpx<double> *>(y + FM);
  double *state = reinterpret_cast<double *>(cvec + F2);
  auto mfac = reinterpret_cast<const cpx<double> *>(state + 4);
  double *z = state + 4 + 12 * 15;
  double *zpart = z + n;
  double *zp = zpart + (size_t)WCH * n;
  double *mpart = zp + (size_t)ZCH * FM * FM;
  // 2D plans: multi-block vector kernels (n = n1^2) and the stencil in the
  // DST-x domain; 1D: single-block kernels with the mass-matrix solve
  const bool mb = p->dims == 2;
  const int NB = fom_vec_blocks(n);
  // two classical Gram-Schmidt passes of w against V rows 0..cnt-1 (T column
  // col, or no T), then (T != NULL) V row cnt = w / ||w||
  auto morth = [&](double *w, int cnt, double *Tc, int col) {
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(fom_mdots_kernel, dim3(NB), dim3(MB), 0, p->stream, n, cnt, p->V, w,
                         mpart);
      hipLaunchKernelGGL(fom_mupdate_kernel, dim3(NB), dim3(MB), 0, p->stream, n, cnt, NB, mpart,
                         p->V, w, Tc, FM, col);
    }
  };
  auto hs = reinterpret_cast<cpx<double> *>(p->fom_h);
  const double s = -1.0 / p->w;
  const int P = (n + 15) / 16;
  if (mb) {
    PD_HIP_CHECK(hipMemsetAsync(T, 0, sizeof(double) * (FM + 1) * FM, p->stream));
    hipLaunchKernelGGL(fom_mdots_kernel, dim3(NB), dim3(MB), 0, p->stream, n, 0, p->V, b, mpart);
    hipLaunchKernelGGL(fom_mscale_kernel, dim3(NB), dim3(MB), 0, p->stream, n, 0, NB, mpart, b,
                       p->V, nullptr, FM, 0, state);
  } else {
    hipLaunchKernelGGL(fom_start_kernel, dim3(1), dim3(FB), 0, p->stream, n, b, p->V, T,
                       (FM + 1) * FM, state);
  }
  PD_HIP_CHECK(hipGetLastError());
  {
    // b = 0 (zero data): x = 0, no Krylov space to build
    double b0 = 0.0;
    PD_HIP_CHECK(hipMemcpyAsync(&b0, state, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
    if (!std::isfinite(b0)) {
      pd_set_error("capacitance right-hand side is not finite");
      return PD_ENONFINITE;
    }
    if (b0 == 0.0) {
      PD_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * n, p->stream));
      if (iters) *iters = 0;
      if (relres) *relres = 0.0;
      if (checks) *checks = 0;
      return PD_OK;
    }
  }
  double beta = 0.0, res = 0.0;
  int m = 0;
  bool checked = false;
  int nchecks = 0;
  while (m < maxm) {
    ++m;
    if (mb) {
      hipLaunchKernelGGL(fom_apply2d_kernel, dim3((n + 255) / 256), dim3(256), 0, p->stream,
                         p->n, p->V + (size_t)(m - 1) * n,
                         p->twd + p->twd_cos, p->uni[3], p->uni[4],
                         p->uni[5], p->wvec);
      morth(p->wvec, m, T, m - 1);
      hipLaunchKernelGGL(fom_mdots_kernel, dim3(NB), dim3(MB), 0, p->stream, n, 0, p->V,
                         p->wvec, mpart);
      hipLaunchKernelGGL(fom_mscale_kernel, dim3(NB), dim3(MB), 0, p->stream, n, m, NB, mpart,
                         p->wvec, p->V, T, FM, m - 1, nullptr);
    } else {
      hipLaunchKernelGGL(fom_apply_kernel, dim3(1), dim3(P), 0, p->stream, n,
                         p->V + (size_t)(m - 1) * n, mfac, p->uni[0], p->uni[2], p->uni[3],
                         p->uni[4], p->uni[5], p->wvec);
      hipLaunchKernelGGL((fom_orth_kernel<FM>), dim3(1), dim3(FB), 0, p->stream, n, m, p->V,
                         p->wvec, T);
    }
    PD_HIP_CHECK(hipGetLastError());
    if (m % q != 0 && m != maxm) continue;
    // h_i for all i: pass C on a zero spectrum with x = v_{m+1} gives -w h_i
    PD_HIP_CHECK(hipMemsetAsync(p->fom_h, 0, p->spec_bytes, p->stream));
    pd_status st = pd_launch_tridiag(p, 1, p->fom_h, p->V + (size_t)m * n, p->fom_h);
    if (st != PD_OK) return st;
    hipLaunchKernelGGL((fom_proj_kernel<FM>),
                       dim3((F2 + PROJ_PT - 1) / PROJ_PT, (m + PROJ_PK - 1) / PROJ_PK), dim3(256),
                       0, p->stream, n, F2, m, hs, p->V, s, proj);
    hipLaunchKernelGGL((fom_small_kernel<FM>), dim3(F2), dim3(64), 0, p->stream, F2, m, p->lam64,
                       p->gB64, p->w, T, proj, Zpart, lastrow);
    hipLaunchKernelGGL((fom_zsum_kernel<FM>), dim3((m * m + 255) / 256, ZCH), dim3(256), 0,
                       p->stream, F2, m, Zpart, zp);
    hipLaunchKernelGGL((fom_solve_kernel<FM>), dim3(1), dim3(FB), 0, p->stream, F2, m, zp,
                       lastrow, p->gB64, state, y, cvec);
    hipLaunchKernelGGL(fom_wsum_kernel, dim3((n + 63) / 64, WCH), dim3(256), 0, p->stream, n, F2,
                       hs, cvec, zpart);
    hipLaunchKernelGGL(fom_wfinish_kernel, dim3((n + 255) / 256), dim3(256), 0, p->stream, n, zpart,
                       s, z);
    if (mb) {
      morth(z, m, nullptr, 0);
      hipLaunchKernelGGL(fom_mdots_kernel, dim3(NB), dim3(MB), 0, p->stream, n, 0, p->V, z,
                         mpart);
      hipLaunchKernelGGL(fom_mres_kernel, dim3(1), dim3(64), 0, p->stream, NB, mpart, T, FM, m,
                         p->w, state);
    } else {
      hipLaunchKernelGGL((fom_resid_kernel<FM>), dim3(1), dim3(FB), 0, p->stream, n, m, p->V, z,
                         T, p->w, state);
    }
    PD_HIP_CHECK(hipGetLastError());
    double hst[2];
    PD_HIP_CHECK(hipMemcpyAsync(hst, state, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
    beta = hst[0];
    res = hst[1];
    checked = true;
    ++nchecks;
    if (!std::isfinite(res) || !std::isfinite(beta)) {
      pd_set_error("Algorithm 2 produced a non-finite residual");
      return PD_ENONFINITE;
    }
    if (res <= rtol * beta) break;
  }
  hipLaunchKernelGGL(fom_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, p->stream, n, m, p->V,
                     y, x);
  PD_HIP_CHECK(hipGetLastError());
  if (iters) *iters = m;
  if (relres) *relres = beta > 0.0 ? res / beta : 0.0;
  if (checks) *checks = nchecks;
  return (checked && res <= rtol * beta) ? PD_OK : PD_ENOTCONV;
}

pd_status pd_fom_apply(pd_plan p, const cpx<double> *mfac, const double *v, double *w) {
  const int n = p->nbar;
  if (n > FB * FR) {
    pd_set_error("Algorithm 2 operator: n exceeds the single-block limit");
    return PD_ENOTSUP;
  }
  hipLaunchKernelGGL(fom_apply_kernel, dim3(1), dim3((n + 15) / 16), 0, p->stream, n, v, mfac,
                     p->uni[0], p->uni[2], p->uni[3], p->uni[4], p->uni[5], w);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// mass factors for fom_apply_kernel (host, float64): 16 rows per thread
void pd_fom_mass_factors(pd_plan p, std::vector<double> &out) {
  out.assign(12 * 15, 0.0);
  pd_partition_factors(p->uni[0], 0.0, p->uni[1], 0.0, p->uni[2], 0.0, 16, out.data());
}

// ---- multi-block vector helpers shared with the block Galerkin method ----

int pd_mvec_blocks(int n) { return fom_vec_blocks(n); }

// Two classical Gram-Schmidt passes of w against V rows 0..cnt-1 (cnt < 40),
// the coefficients added to T[k * ldT + col] (T may be NULL).  part holds
// pd_mvec_blocks(n) * 40 doubles.
pd_status pd_mvec_orth(pd_plan p, int n, const double *V, double *w, int cnt, double *T, int ldT,
                       int col, double *part) {
  if (cnt >= MCAP) {
    pd_set_error("multi-block orthogonalisation: too many basis vectors");
    return PD_EINVAL;
  }
  const int NB = fom_vec_blocks(n);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(fom_mdots_kernel, dim3(NB), dim3(MB), 0, p->stream, n, cnt, V, w, part);
    hipLaunchKernelGGL(fom_mupdate_kernel, dim3(NB), dim3(MB), 0, p->stream, n, cnt, NB, part, V,
                       w, T, ldT, col);
  }
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// V row cnt = w / ||w||; ||w|| written to T[cnt * ldT + col] (T != NULL) and
// *tout (tout != NULL).
pd_status pd_mvec_normalize(pd_plan p, int n, double *V, const double *w, int cnt, double *T,
                            int ldT, int col, double *tout, double *part) {
  const int NB = fom_vec_blocks(n);
  hipLaunchKernelGGL(fom_mdots_kernel, dim3(NB), dim3(MB), 0, p->stream, n, 0, V, w, part);
  hipLaunchKernelGGL(fom_mscale_kernel, dim3(NB), dim3(MB), 0, p->stream, n, cnt, NB, part, w, V,
                     T, ldT, col, tout);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// out[0] = (acc ? out[0] : 0) + w . w
pd_status pd_mvec_norm2(pd_plan p, int n, const double *w, double *out, int acc, double *part) {
  const int NB = fom_vec_blocks(n);
  hipLaunchKernelGGL(fom_mdots_kernel, dim3(NB), dim3(MB), 0, p->stream, n, 0, w, w, part);
  hipLaunchKernelGGL(fom_maccum_kernel, dim3(1), dim3(64), 0, p->stream, NB, part, acc, out);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// 2D plans: w = tau K v in the DST-x domain of the line solves
pd_status pd_apply2d(pd_plan p, const double *v, double *w) {
  const int n = p->nbar;
  hipLaunchKernelGGL(fom_apply2d_kernel, dim3((n + 255) / 256), dim3(256), 0, p->stream, p->n, v,
                     p->twd + p->twd_cos, p->uni[3], p->uni[4],
                     p->uni[5], w);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}
