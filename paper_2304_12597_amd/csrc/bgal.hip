// The block Galerkin method for the BDF capacitance system J^(s) x = b^(s)
// (Section 5, Proposition), on the GPU.
//
// Block Arnoldi on A = tau beta M^{-1} K (P_i^{-1} M = (nu_i I + A)^{-1},
// nu_i = 1 - pi_i; for M = I the paper's tau beta K) from the starting block
// B = [b_1 .. b_s] = V_1 beta, column by column: the j-th column of the new
// block is A applied to column j of the current block, orthogonalised
// against every basis vector so far (two classical Gram-Schmidt passes), so
// that A V_m = V_m T_m + V_{m+1} t_{m+1,m} E_m^T with t_{m+1,m} upper
// triangular.  x_k = V_m y_k with y from (I + T) y = (e_1 (x) I_s) beta,
//   T_{k,h} = sum_i gamma_i^(k) theta_i^(h) E_i,
//   E_i = S_i - V_m^T H_i t_{m+1,m} E_m^T S_i,
//   S_i = (nu_i I + T_m)^{-1},  H_i = P_i^{-1} M V_{m+1},
// and the residual norm of the Proposition,
//   ||r||^2 = sum_k ||(I - V_m V_m^T) sum_i gamma_i^(k) H_i t_{m+1,m}
//             E_m^T S_i sum_h theta_i^(h) y_h||^2.
// The sums over the full spectrum use its conjugate halves (weights 1 at
// i = 0 and ell/2, 2 elsewhere, real part).  Each check is one parfor of
// shifted solves with s right-hand sides per frequency (s launches of the
// pass-C kernel on a zero spectrum, which writes -h).  The basis dimension
// s m is at most BG_SMAX and at most n (where the block space is all of R^n).
#include "pd_internal.h"
#include "pd_gj.h"
#include "pd_proj.h"

#include <cmath>
#include <vector>

namespace {

constexpr int FB = 512;          // single-block kernels
constexpr int FR = 16;           // rows per thread of the single-block kernels
constexpr int CAP = 40;          // basis vectors an orthogonalisation handles (>= SMAX + 5)
constexpr int NCH = 16;          // frequency chunks of the Galerkin-matrix sums
constexpr int SMX = BG_SMAX;
constexpr int NMAX = 6 * SMX;    // largest Galerkin system
using Cx = cpx<double>;

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

// Two classical Gram-Schmidt passes of w against V rows 0..cnt-1:
// T[k*ldT + col] += dots (k < cnt), T[cnt*ldT + col] = ||w'||, V row cnt =
// w' / ||w'|| (0 if w' = 0).  cnt < CAP.
__global__ void __launch_bounds__(FB)
bg_orth_kernel(int n, int cnt, int col, int ldT, double *__restrict__ V,
               const double *__restrict__ wsrc, double *__restrict__ T) {
  __shared__ double red[FB / 64];
  __shared__ double part[CAP][FB / 64];
  __shared__ double dots[CAP];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63, nw = FB / 64;
  double wv[FR];
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int i = tid + r * FB;
    wv[r] = i < n ? wsrc[i] : 0.0;
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int k = 0; k < cnt; ++k) {
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
    if (tid < cnt) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += part[tid][q];
      dots[tid] = s;
      T[(size_t)tid * ldT + col] += s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const int i = tid + r * FB;
      if (i < n)
        for (int k = 0; k < cnt; ++k) wv[r] -= dots[k] * V[(size_t)k * n + i];
    }
    __syncthreads();
  }
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < FR; ++r) s += wv[r] * wv[r];
  const double t = sqrt(block_sum(s, red));
  if (tid == 0) T[(size_t)cnt * ldT + col] = t;
#pragma unroll
  for (int r = 0; r < FR; ++r) {
    const int i = tid + r * FB;
    if (i < n) V[(size_t)cnt * n + i] = t > 0.0 ? wv[r] / t : 0.0;
  }
}

// proj[i][k][j] = (V_k . h_i^(j)) for k < sm, j < s (hs_j holds -h^(j),
// spectra `sstride` complex elements apart).  Grid: (ceil(F2 / PROJ_PT),
// ceil(sm / PROJ_PK), s) tiles.
__global__ void __launch_bounds__(256)
bg_proj_kernel(int n, int F2, int sm, const Cx *__restrict__ hs, size_t sstride,
               const double *__restrict__ V, Cx *__restrict__ proj) {
  const int i0 = blockIdx.x * PROJ_PT, k0 = blockIdx.y * PROJ_PK, j = blockIdx.z;
  Cx v;
  proj_tile(n, F2, sm, V, hs + j * sstride, i0, k0, v);
  const int t = threadIdx.x;
  if (t < PROJ_PK * PROJ_PT) {
    const int k = k0 + t / PROJ_PT, i = i0 + t % PROJ_PT;
    if (k < sm && i < F2) proj[((size_t)i * SMX + k) * 6 + j] = Cx{-v.re, -v.im};
  }
}

// One wave per frequency i: S_i = (nu_i I + T_m)^{-1} by Gauss-Jordan in LDS
// (wave_gj_inverse); L_i = the last s rows of S_i (E_m^T S_i);
// E_i = S_i - proj_i t_{m+1,m} L_i.  Lane c writes column c.
__global__ void __launch_bounds__(64)
bg_small_kernel(int F2, int sm, int s, int m, const double *__restrict__ lam,
                const double *__restrict__ T, int ldT, const Cx *__restrict__ proj,
                Cx *__restrict__ E, Cx *__restrict__ L) {
  __shared__ Cx a[SMX][2 * SMX];
  __shared__ Cx fcol[SMX];
  const int i = blockIdx.x, c = threadIdx.x;
  wave_gj_inverse<SMX>(sm, Cx{lam[2 * i], lam[2 * i + 1]}, T, ldT, a, fcol);
  if (c >= sm) return;
  Cx *Li = L + (size_t)i * 6 * SMX;
  Cx lc[6];
  for (int q = 0; q < s; ++q) {
    lc[q] = a[sm - s + q][sm + c];
    Li[q * SMX + c] = lc[q];
  }
  // t_{m+1,m}: rows sm..sm+s-1, columns (m-1)s..ms-1 of T (upper triangular)
  const int c0 = (m - 1) * s;
  Cx *Ei = E + (size_t)i * SMX * SMX;
  for (int r = 0; r < sm; ++r) {
    Cx e = a[r][sm + c];
    for (int q = 0; q < s; ++q) {       // (proj_i t)_{r,q} L_i[q][c]
      Cx pq = {0.0, 0.0};
      for (int j = 0; j <= q; ++j) {
        const double t = T[(size_t)(sm + j) * ldT + c0 + q];
        const Cx pv = proj[((size_t)i * SMX + r) * 6 + j];
        pq.re += pv.re * t;
        pq.im += pv.im * t;
      }
      e = csub(e, cmul(pq, lc[q]));
    }
    Ei[r * SMX + c] = e;
  }
}

// part[ch][(k s + h)][r][c] = sum over chunk ch of frequencies of
// Re(ctab[k s + h][i] E_i[r][c]).  Grid: (ceil(sm^2/256), NCH).
__global__ void __launch_bounds__(256)
bg_assemble_kernel(int F2, int sm, int s, const Cx *__restrict__ ctab,
                   const Cx *__restrict__ E, double *__restrict__ part) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int ch = blockIdx.y;
  if (e >= sm * sm) return;
  const int r = e / sm, c = e - r * sm;
  const int per = (F2 + NCH - 1) / NCH;
  const int i0 = ch * per, i1 = (i0 + per < F2) ? i0 + per : F2;
  double acc[36];
  for (int q = 0; q < 36; ++q) acc[q] = 0.0;
  for (int i = i0; i < i1; ++i) {
    const Cx ev = E[(size_t)i * SMX * SMX + r * SMX + c];
    for (int q = 0; q < s * s; ++q) {
      const Cx w = ctab[(size_t)q * F2 + i];
      acc[q] += w.re * ev.re - w.im * ev.im;
    }
  }
  for (int q = 0; q < s * s; ++q)
    part[(((size_t)ch * 36 + q) * SMX + r) * SMX + c] = acc[q];
}

// G = I + sum of the chunk partials, rhs = (e_1 (x) I_s) beta per block,
// y = G^{-1} rhs by Gaussian elimination with partial pivoting (G in the
// global scratch, ld N + 1).  One block.
__global__ void __launch_bounds__(256)
bg_solve_kernel(int sm, int s, const double *__restrict__ part, const double *__restrict__ beta,
                double *__restrict__ G, double *__restrict__ y) {
  __shared__ int piv_s;
  __shared__ double ys[NMAX];
  const int N = s * sm, ld = N + 1, tid = threadIdx.x;
  for (int e = tid; e < N * N; e += 256) {
    const int row = e / N, col = e - row * N;
    const int k = row / sm, r = row - k * sm, h = col / sm, c = col - h * sm;
    double v = (row == col) ? 1.0 : 0.0;
    for (int ch = 0; ch < NCH; ++ch)
      v += part[(((size_t)ch * 36 + k * s + h) * SMX + r) * SMX + c];
    G[(size_t)row * ld + col] = v;
  }
  for (int row = tid; row < N; row += 256) {
    const int k = row / sm, r = row - k * sm;
    G[(size_t)row * ld + N] = (r < s) ? beta[r * 6 + k] : 0.0;
  }
  __syncthreads();
  __shared__ double wmag[4];
  __shared__ int widx[4];
  for (int col = 0; col < N; ++col) {
    // pivot: the first row r >= col with the largest |G[r][col]| (one row
    // per thread, N <= 256; wave argmax by shuffles, then over the waves)
    double mag = -1.0;
    int idx = tid;
    if (tid >= col && tid < N) mag = fabs(G[(size_t)tid * ld + col]);
    for (int off = 32; off > 0; off >>= 1) {
      const double om = __shfl_xor(mag, off, 64);
      const int oi = __shfl_xor(idx, off, 64);
      if (om > mag || (om == mag && oi < idx)) {
        mag = om;
        idx = oi;
      }
    }
    if ((tid & 63) == 0) {
      wmag[tid >> 6] = mag;
      widx[tid >> 6] = idx;
    }
    __syncthreads();
    if (tid == 0) {
      int p = widx[0];
      double best = wmag[0];
      for (int w = 1; w < 4; ++w)
        if (wmag[w] > best) {
          best = wmag[w];
          p = widx[w];
        }
      piv_s = p;
    }
    __syncthreads();
    const int p = piv_s;
    if (p != col)
      for (int c = col + tid; c <= N; c += 256) {
        const double t = G[(size_t)col * ld + c];
        G[(size_t)col * ld + c] = G[(size_t)p * ld + c];
        G[(size_t)p * ld + c] = t;
      }
    __syncthreads();
    const double dinv = 1.0 / G[(size_t)col * ld + col];
    for (int r = col + 1 + tid; r < N; r += 256) {
      const double f = G[(size_t)r * ld + col] * dinv;
      for (int c = col + 1; c <= N; ++c) G[(size_t)r * ld + c] -= f * G[(size_t)col * ld + c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int r = N - 1; r >= 0; --r) {
      double v = G[(size_t)r * ld + N];
      for (int c = r + 1; c < N; ++c) v -= G[(size_t)r * ld + c] * ys[c];
      ys[r] = v / G[(size_t)r * ld + r];
    }
  }
  __syncthreads();
  for (int r = tid; r < N; r += 256) y[r] = ys[r];
}

// One thread per frequency: u = sum_h theta_i^(h) y_h, v = L_i u,
// w = t_{m+1,m} v, cw[i][k][j] = gtab[k][i] w_j.
__global__ void __launch_bounds__(64)
bg_cw_kernel(int F2, int sm, int s, int m, const Cx *__restrict__ L,
             const double *__restrict__ T, int ldT, const Cx *__restrict__ thtab,
             const Cx *__restrict__ gtab, const double *__restrict__ y, Cx *__restrict__ cw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F2) return;
  const Cx *Li = L + (size_t)i * 6 * SMX;
  Cx v[6];
  for (int q = 0; q < s; ++q) v[q] = Cx{0.0, 0.0};
  for (int c = 0; c < sm; ++c) {
    Cx u = {0.0, 0.0};
    for (int h = 0; h < s; ++h) {
      const Cx th = thtab[(size_t)h * F2 + i];
      const double yv = y[h * sm + c];
      u.re += th.re * yv;
      u.im += th.im * yv;
    }
    for (int q = 0; q < s; ++q) {
      const Cx l = Li[q * SMX + c];
      v[q].re += l.re * u.re - l.im * u.im;
      v[q].im += l.re * u.im + l.im * u.re;
    }
  }
  const int c0 = (m - 1) * s;
  Cx w[6];
  for (int j = 0; j < s; ++j) {
    Cx acc = {0.0, 0.0};
    for (int q = j; q < s; ++q) {
      const double t = T[(size_t)(sm + j) * ldT + c0 + q];
      acc.re += t * v[q].re;
      acc.im += t * v[q].im;
    }
    w[j] = acc;
  }
  for (int k = 0; k < s; ++k) {
    const Cx g = gtab[(size_t)k * F2 + i];
    for (int j = 0; j < s; ++j) cw[((size_t)i * 6 + k) * 6 + j] = cmul(g, w[j]);
  }
}

// zpart[ch][k][row] = -sum over the ch-th chunk of frequencies i of
// sum_j Re(cw[i][k][j] h_i^(j)[row]) (hs_j = -h^(j)).  Block: 64 rows x 4
// frequency lanes; grid (ceil(n/64), NCH).
__global__ void __launch_bounds__(256)
bg_wsum_kernel(int n, int F2, int s, const Cx *__restrict__ hs, size_t sstride,
               const Cx *__restrict__ cw, double *__restrict__ zpart) {
  __shared__ double sh[4][6][64];
  const int col = threadIdx.x & 63, lane = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + col, ch = blockIdx.y;
  const int per = (F2 + NCH - 1) / NCH;
  const int i0 = ch * per, i1 = (i0 + per < F2) ? i0 + per : F2;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (row < n)
    for (int i = i0 + lane; i < i1; i += 4)
      for (int j = 0; j < s; ++j) {
        const Cx h = hs[j * sstride + (size_t)i * n + row];
#pragma unroll
        for (int k = 0; k < 6; ++k)
          if (k < s) {
            const Cx c = cw[((size_t)i * 6 + k) * 6 + j];
            acc[k] -= c.re * h.re - c.im * h.im;
          }
      }
#pragma unroll
  for (int k = 0; k < 6; ++k) sh[lane][k][col] = acc[k];
  __syncthreads();
  if (lane == 0 && row < n)
    for (int k = 0; k < s; ++k)
      zpart[((size_t)ch * 6 + k) * n + row] =
          sh[0][k][col] + sh[1][k][col] + sh[2][k][col] + sh[3][k][col];
}

// z[k][row] = sum_ch zpart[ch][k][row] (fixed order).  Grid (ceil(n/256), s).
__global__ void __launch_bounds__(256)
bg_wfinish_kernel(int n, const double *__restrict__ zpart, double *__restrict__ z) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (row >= n) return;
  double acc = 0.0;
  for (int ch = 0; ch < NCH; ++ch) acc += zpart[((size_t)ch * 6 + k) * n + row];
  z[(size_t)k * n + row] = acc;
}

// state[1] = sqrt(sum_k ||(I - V V^T) z_k||^2) (two projection passes).
__global__ void __launch_bounds__(FB)
bg_resid_kernel(int n, int sm, int s, const double *__restrict__ V, const double *__restrict__ z,
                double *__restrict__ state) {
  __shared__ double red[FB / 64];
  __shared__ double part[SMX][FB / 64];
  __shared__ double dots[SMX];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63, nw = FB / 64;
  double total = 0.0;
  for (int k = 0; k < s; ++k) {
    double zv[FR];
#pragma unroll
    for (int r = 0; r < FR; ++r) {
      const int i = tid + r * FB;
      zv[r] = i < n ? z[(size_t)k * n + i] : 0.0;
    }
    for (int pass = 0; pass < 2; ++pass) {
      for (int c = 0; c < sm; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < FR; ++r) {
          const int i = tid + r * FB;
          if (i < n) sacc += V[(size_t)c * n + i] * zv[r];
        }
        for (int off = 32; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
        if (lane == 0) part[c][wid] = sacc;
      }
      __syncthreads();
      if (tid < sm) {
        double a = 0.0;
        for (int q = 0; q < nw; ++q) a += part[tid][q];
        dots[tid] = a;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < FR; ++r) {
        const int i = tid + r * FB;
        if (i < n)
          for (int c = 0; c < sm; ++c) zv[r] -= dots[c] * V[(size_t)c * n + i];
      }
      __syncthreads();
    }
    double sq = 0.0;
#pragma unroll
    for (int r = 0; r < FR; ++r) sq += zv[r] * zv[r];
    total += block_sum(sq, red);
  }
  if (tid == 0) state[1] = sqrt(total);
}

// x[k n + row] = sum_c y[k sm + c] V[c][row]
__global__ void __launch_bounds__(256)
bg_combine_kernel(int n, int sm, int s, const double *__restrict__ V,
                  const double *__restrict__ y, double *__restrict__ x) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (row >= n || k >= s) return;
  double acc = 0.0;
  for (int c = 0; c < sm; ++c) acc += y[k * sm + c] * V[(size_t)c * n + row];
  x[(size_t)k * n + row] = acc;
}

// out[0] = sqrt(in[0])
__global__ void bg_sqrt_kernel(const double *__restrict__ in, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = sqrt(in[0]);
}

// ||b||^2 of the s starting vectors into state[0] (as a norm)
__global__ void __launch_bounds__(FB)
bg_norm_kernel(int len, const double *__restrict__ b, double *__restrict__ state) {
  __shared__ double red[FB / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < len; i += FB) s += b[i] * b[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) state[0] = sqrt(s);
}

}  // namespace

// Layout of the block Galerkin state (doubles), F2 frequencies, n rows.
BgLayout pd_bgal_layout(int n, int F2) {
  BgLayout L;
  size_t o = 0;
  auto take = [&](size_t cnt) {
    const size_t at = o;
    o += (cnt + 1) & ~(size_t)1;   // keep complex arrays 16-byte aligned
    return at;
  };
  L.T = take((size_t)BG_TROWS * BG_LDT);
  L.beta = take(36);
  L.proj = take(2 * (size_t)F2 * SMX * 6);
  L.E = take(2 * (size_t)F2 * SMX * SMX);
  L.L = take(2 * (size_t)F2 * 6 * SMX);
  L.part = take((size_t)NCH * 36 * SMX * SMX);
  L.G = take((size_t)NMAX * (NMAX + 1));
  L.y = take(NMAX);
  L.cw = take(2 * (size_t)F2 * 36);
  L.z = take(6 * (size_t)n);
  L.zpart = take((size_t)NCH * 6 * n);
  L.state = take(8);
  L.mpart = take((size_t)256 * 40);
  L.mfac = take(12 * 15);
  L.ctab = take(2 * (size_t)36 * F2);
  L.gtab = take(2 * (size_t)6 * F2);
  L.thtab = take(2 * (size_t)6 * F2);
  L.total = o;
  return L;
}

pd_status pd_bgal(pd_plan p, const double *b, double *x, double rtol, int *iters,
                  double *relres, int *checks) {
  const int n = p->nbar, F2 = p->F2, s = p->bdf_s;
  // 1D: single-block vector kernels (n <= FB * FR); 2D: multi-block ones,
  // the vectors in the DST-x domain of the line solves
  const bool mb = p->dims == 2;
  if (s < 1 || s > 6 || (!mb && n > FB * FR) || !p->fom || !p->fom_h) {
    pd_set_error("block Galerkin: unsupported plan");
    return PD_ENOTSUP;
  }
  const BgLayout Lo = pd_bgal_layout(n, F2);
  double *base = p->fom;
  double *T = base + Lo.T;
  double *beta = base + Lo.beta;
  Cx *proj = reinterpret_cast<Cx *>(base + Lo.proj);
  Cx *E = reinterpret_cast<Cx *>(base + Lo.E);
  Cx *Lr = reinterpret_cast<Cx *>(base + Lo.L);
  double *part = base + Lo.part;
  double *G = base + Lo.G;
  double *y = base + Lo.y;
  Cx *cw = reinterpret_cast<Cx *>(base + Lo.cw);
  double *z = base + Lo.z;
  double *zpart = base + Lo.zpart;
  double *state = base + Lo.state;
  double *mpart = base + Lo.mpart;
  const Cx *mfac = reinterpret_cast<const Cx *>(base + Lo.mfac);
  const Cx *ctab = reinterpret_cast<const Cx *>(base + Lo.ctab);
  const Cx *gtab = reinterpret_cast<const Cx *>(base + Lo.gtab);
  const Cx *thtab = reinterpret_cast<const Cx *>(base + Lo.thtab);
  Cx *hs = reinterpret_cast<Cx *>(p->fom_h);
  const size_t sstride = (size_t)F2 * n;   // complex elements per spectrum
  int mmax = SMX / s;
  if (p->maxit < mmax) mmax = p->maxit;
  if (n / s < mmax) mmax = n / s;          // the basis spans R^n at s m = n
  if (mmax < 1) {
    pd_set_error("block Galerkin: n < s");
    return PD_ENOTSUP;
  }
  const int q = p->fom_q < 1 ? 1 : p->fom_q;
  double *V = p->V;                        // (maxit + 1) * s * n >= (mmax + 1) * s * n

  PD_HIP_CHECK(hipMemsetAsync(T, 0, sizeof(double) * BG_TROWS * BG_LDT, p->stream));
  PD_HIP_CHECK(hipMemsetAsync(beta, 0, sizeof(double) * 36, p->stream));
  if (mb) {
    pd_status st = pd_mvec_norm2(p, s * n, b, state + 2, 0, mpart);
    if (st != PD_OK) return st;
    hipLaunchKernelGGL(bg_sqrt_kernel, dim3(1), dim3(64), 0, p->stream, state + 2, state);
  } else {
    hipLaunchKernelGGL(bg_norm_kernel, dim3(1), dim3(FB), 0, p->stream, s * n, b, state);
  }
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
      PD_HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * (size_t)s * n, p->stream));
      if (iters) *iters = 0;
      if (relres) *relres = 0.0;
      if (checks) *checks = 0;
      return PD_OK;
    }
  }
  // B = V_1 beta (Gram-Schmidt QR of the s starting columns, beta ld 6;
  // the multi-block form orthogonalises b in place)
  for (int j = 0; j < s; ++j) {
    if (mb) {
      double *bj = const_cast<double *>(b) + (size_t)j * n;
      pd_status st = pd_mvec_orth(p, n, V, bj, j, beta, 6, j, mpart);
      if (st == PD_OK) st = pd_mvec_normalize(p, n, V, bj, j, beta, 6, j, nullptr, mpart);
      if (st != PD_OK) return st;
    } else {
      hipLaunchKernelGGL(bg_orth_kernel, dim3(1), dim3(FB), 0, p->stream, n, j, j, 6, V,
                         b + (size_t)j * n, beta);
    }
  }
  PD_HIP_CHECK(hipGetLastError());
  double bnorm = 0.0, res = 0.0;
  int m = 0, nchecks = 0;
  bool checked = false;
  while (m < mmax) {
    ++m;
    const int sm = s * m;
    for (int j = 0; j < s; ++j) {
      const double *vj = V + (size_t)((m - 1) * s + j) * n;
      const int col = (m - 1) * s + j;
      if (mb) {
        pd_status st = pd_apply2d(p, vj, p->wvec);
        if (st == PD_OK) st = pd_mvec_orth(p, n, V, p->wvec, sm + j, T, BG_LDT, col, mpart);
        if (st == PD_OK)
          st = pd_mvec_normalize(p, n, V, p->wvec, sm + j, T, BG_LDT, col, nullptr, mpart);
        if (st != PD_OK) return st;
      } else {
        pd_status st = pd_fom_apply(p, mfac, vj, p->wvec);
        if (st != PD_OK) return st;
        hipLaunchKernelGGL(bg_orth_kernel, dim3(1), dim3(FB), 0, p->stream, n, sm + j, col,
                           BG_LDT, V, p->wvec, T);
      }
    }
    PD_HIP_CHECK(hipGetLastError());
    if (m % q != 0 && m != mmax) continue;
    // H_i for all i: pass C on a zero spectrum with x = column j of V_{m+1}
    for (int j = 0; j < s; ++j) {
      Cx *hj = hs + j * sstride;
      PD_HIP_CHECK(hipMemsetAsync(hj, 0, sstride * sizeof(Cx), p->stream));
      pd_status st = pd_launch_tridiag(p, 1, hj, V + (size_t)(sm + j) * n, hj);
      if (st != PD_OK) return st;
    }
    hipLaunchKernelGGL(bg_proj_kernel,
                       dim3((F2 + PROJ_PT - 1) / PROJ_PT, (sm + PROJ_PK - 1) / PROJ_PK, s),
                       dim3(256), 0, p->stream, n, F2, sm, hs, sstride, V, proj);
    hipLaunchKernelGGL(bg_small_kernel, dim3(F2), dim3(64), 0, p->stream, F2, sm, s, m, p->lam64,
                       T, BG_LDT, proj, E, Lr);
    hipLaunchKernelGGL(bg_assemble_kernel, dim3((sm * sm + 255) / 256, NCH), dim3(256), 0,
                       p->stream, F2, sm, s, ctab, E, part);
    hipLaunchKernelGGL(bg_solve_kernel, dim3(1), dim3(256), 0, p->stream, sm, s, part, beta, G,
                       y);
    hipLaunchKernelGGL(bg_cw_kernel, dim3((F2 + 63) / 64), dim3(64), 0, p->stream, F2, sm, s, m,
                       Lr, T, BG_LDT, thtab, gtab, y, cw);
    hipLaunchKernelGGL(bg_wsum_kernel, dim3((n + 63) / 64, NCH), dim3(256), 0, p->stream, n, F2,
                       s, hs, sstride, cw, zpart);
    hipLaunchKernelGGL(bg_wfinish_kernel, dim3((n + 255) / 256, s), dim3(256), 0, p->stream, n,
                       zpart, z);
    if (mb) {
      for (int k = 0; k < s; ++k) {
        pd_status st = pd_mvec_orth(p, n, V, z + (size_t)k * n, sm, nullptr, 0, 0, mpart);
        if (st == PD_OK) st = pd_mvec_norm2(p, n, z + (size_t)k * n, state + 2, k > 0, mpart);
        if (st != PD_OK) return st;
      }
      hipLaunchKernelGGL(bg_sqrt_kernel, dim3(1), dim3(64), 0, p->stream, state + 2, state + 1);
    } else {
      hipLaunchKernelGGL(bg_resid_kernel, dim3(1), dim3(FB), 0, p->stream, n, sm, s, V, z,
                         state);
    }
    PD_HIP_CHECK(hipGetLastError());
    double hst[2];
    PD_HIP_CHECK(hipMemcpyAsync(hst, state, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    PD_HIP_CHECK(hipStreamSynchronize(p->stream));
    bnorm = hst[0];
    res = hst[1];
    checked = true;
    ++nchecks;
    if (!std::isfinite(res) || !std::isfinite(bnorm)) {
      pd_set_error("block Galerkin produced a non-finite residual");
      return PD_ENONFINITE;
    }
    if (res <= rtol * bnorm) break;
  }
  const int sm = s * m;
  hipLaunchKernelGGL(bg_combine_kernel, dim3((n + 255) / 256, s), dim3(256), 0, p->stream, n, sm,
                     s, V, y, x);
  PD_HIP_CHECK(hipGetLastError());
  if (iters) *iters = m;
  if (relres) *relres = bnorm > 0.0 ? res / bnorm : 0.0;
  if (checks) *checks = nchecks;
  return (checked && res <= rtol * bnorm) ? PD_OK : PD_ENOTCONV;
}
