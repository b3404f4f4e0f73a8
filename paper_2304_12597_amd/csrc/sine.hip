// Shifted solves in the sine basis, for symmetric Toeplitz M and K with zero
// Dirichlet ends (uniform 1D grids; Section 6.1 uses the same basis along x
// for the 2D Laplacian).  The orthonormal DST-I S (S = S^T = S^{-1})
// diagonalises both: M = S diag(m) S, tau K = S diag(kap) S with
// m_k = m_d + 2 m_o cos(pi k/(n+1)), kap_k = tau (k_d + 2 k_o cos(pi k/(n+1))).
// In that basis every step of Algorithm 1 acts mode by mode:
//   P_j^{-1} M            -> m_k / (lambda_j m_k + kap_k)
//   J_ell                 -> phi_k = 1 + w sum_j gamma_j m_k / (lambda_j m_k + kap_k)
// so the capacitance system is diagonal and solved exactly (x_k = b_k/phi_k),
// and a solve is: DST of every time row, one kernel per tile of modes (time
// DFT, the per-mode solve with its SMW correction, inverse time DFT), DST of
// every time row again.
//
// DST-I of a row x_1..x_{N-1} (N = n+1 a power of two) from one complex FFT
// of length H = N/2: with x_0 = x_N = 0 form
//   y_j = sin(pi j/N) (x_j + x_{N-j}) + (x_j - x_{N-j})/2,  j = 0..N-1,
// take its real DFT Y_m = R_m - i I_m (from the complex FFT of
// y_{2m} + i y_{2m+1} and the usual even/odd split), then
//   S_{2m} = I_m,  S_{2m+1} = R_0/2 + R_1 + ... + R_m
// (the odd outputs are a prefix sum, done as a block scan).
#include "pd_internal.h"
#include "pd_fft.h"

#include <cmath>

namespace {

using namespace pdfft;

// C rows per block, H/8 threads per row, each owning 8 consecutive m.
// MODE 0: rows h_t = tau f_t (+ u0 at t = 0); MODE 1: rows of `in`.
// out may alias in (every row is read completely before it is written).
// LDS: [C * stride cpx columns][twiddles of length H][T double scan sums]
// (at most 128 VGPRs: two 512-thread blocks per CU)
template <int MODE>
__global__ void __launch_bounds__(512, 4)
dst_rows_kernel(int n, int C, int stride, double tau, const double *__restrict__ u0,
                const double *__restrict__ F, const double *in,
                const double *__restrict__ sinq, const cpx<double> *__restrict__ wN,
                const cpx<double> *__restrict__ twH, double *out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using Cx = cpx<double>;
  Cx *lds = reinterpret_cast<Cx *>(smem_raw);
  const int N = n + 1, H = N / 2;
  Cx *twl = lds + C * stride;
  double *scan = reinterpret_cast<double *>(twl + pd_tw_entries(H));
  tw_to_lds(twl, twH, H);
  const int tid = threadIdx.x;
  const int lgG = __builtin_ctz(H) - 3;        // threads per row: G = H/8
  const int G = 1 << lgG;
  const int c = tid >> lgG, lt = tid & (G - 1);
  const int row = blockIdx.x * C + c;
  const size_t base = (size_t)row * n;
  auto xval = [&](int j) -> double {          // x_j, j = 0..N; zero at both ends
    const int i = j - 1;
    const int ic = i < 0 ? 0 : (i >= n ? n - 1 : i);
    double v;
    if constexpr (MODE == 0) {
      v = tau * F[base + ic];
      if (row == 0) v += u0[ic];
    } else {
      v = in[base + ic];
    }
    return (i >= 0 && i < n) ? v : 0.0;
  };
  Cx *col = lds + c * stride;
  // packed input c_m = y_{2m} + i y_{2m+1}, m = lt + u G: consecutive lanes
  // read neighbouring elements; real parts, then imaginary parts (16 loads
  // in flight per phase)
  double *cold = reinterpret_cast<double *>(col);
#pragma unroll
  for (int ph = 0; ph < 2; ++ph) {
    double xa[8], xb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = 2 * (lt + u * G) + ph;
      xa[u] = xval(j);
      xb[u] = xval(N - j);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = lt + u * G;
      const int j = 2 * m + ph;
      cold[2 * pd_fpad(m) + ph] = sinq[j] * (xa[u] + xb[u]) + 0.5 * (xa[u] - xb[u]);
    }
  }
  __syncthreads();
  fft_lds<double, false>(lds, H, C, stride, twl);
  // split the packed real transform: Y_m = E_m + exp(-2 pi i m/N) O_m
  double Rv[8], Iv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int m = 8 * lt + u;
    const Cx a = col[pd_fpad(m)];
    const Cx b = col[pd_fpad((H - m) & (H - 1))];
    const Cx E = {0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
    const Cx O = {0.5 * (a.im + b.im), 0.5 * (b.re - a.re)};
    const Cx w = wN[m];
    Rv[u] = E.re + (w.re * O.re - w.im * O.im);
    Iv[u] = -(E.im + (w.re * O.im + w.im * O.re));
  }
  // odd outputs: inclusive prefix sum of R'_0 = R_0/2, R'_m = R_m
  if (lt == 0) Rv[0] *= 0.5;
  double loc[8];
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    s += Rv[u];
    loc[u] = s;
  }
  // prefix over the row's threads: within the wave by shuffles (segments of
  // G lanes when a wave holds several rows), then over the row's waves
  const int lane = tid & 63, seg = G < 64 ? G : 64;
  double incl = s;
  for (int off = 1; off < seg; off <<= 1) {
    const double v = __shfl_up(incl, off, 64);
    if ((lane & (seg - 1)) >= off) incl += v;
  }
  if (G > 64) {
    if (lane == 63) scan[tid >> 6] = incl;
    __syncthreads();
    const int w0 = (tid >> 6) & ~((G >> 6) - 1);   // first wave of this row
    for (int q = w0; q < (tid >> 6); ++q) incl += scan[q];
  }
  const double excl = incl - s;
  // results in row order through LDS (every thread has finished its split
  // reads), then contiguous stores
  double *orow = reinterpret_cast<double *>(col);
  const double scale = sqrt(2.0 / (double)N);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int m = 8 * lt + u;
    // S_{2m} (m >= 1) at output index 2m - 1, S_{2m+1} at 2m
    if (m >= 1) orow[2 * m - 1] = scale * Iv[u];
    orow[2 * m] = scale * (excl + loc[u]);
  }
  __syncthreads();
  const int T = blockDim.x;
  for (int idx = tid; idx < C * n; idx += T) {
    const int rc = idx / n, i = idx - rc * n;
    const double *src = reinterpret_cast<const double *>(lds + rc * stride);
    out[(size_t)(blockIdx.x * C + rc) * n + i] = src[i];
  }
}

// One tile of 2C consecutive modes over all ell time steps: forward time DFT
// (two real columns per complex column, as in the time transforms), the
// per-mode solve with its exact capacitance correction, inverse time DFT.
// A, B: [ell][n] float64 (the DST coefficients of h and of U).
// LDS: [C * stride cpx][twiddles][2 * nwaves * S double sums]
__global__ void __launch_bounds__(512)
sine_modal_kernel(int N, int n, int C, int stride, const double *__restrict__ A,
                  const double *__restrict__ dal, const cpx<double> *__restrict__ tw,
                  const double *__restrict__ mk, const double *__restrict__ kk, double w,
                  double *__restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using Cx = cpx<double>;
  Cx *lds = reinterpret_cast<Cx *>(smem_raw);
  Cx *twl = lds + C * stride;
  const int T = blockDim.x, tid = threadIdx.x;
  const int nw = T >> 6;
  const int lgS = __builtin_ctz(C) + 1, S = 2 * C;
  double *sb = reinterpret_cast<double *>(twl + pd_tw_entries(N));
  double *sf = sb + nw * S;
  tw_to_lds(twl, tw, N);
  const int tile = blockIdx.x;
  const int i0 = tile * S;
  const int pnt = tid & (S - 1);
  const int t0 = tid >> lgS, dt = T >> lgS;
  const int mode = i0 + pnt;
  const bool inb = mode < n;
  const int mc = inb ? mode : n - 1;
  double *lcol = reinterpret_cast<double *>(lds + (pnt >> 1) * stride) + (pnt & 1);
  const double *dalinv = dal ? dal + N : nullptr;
  for (int tb = t0; tb < N; tb += 8 * dt) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = tb + u * dt;
      const int tc = t < N ? t : N - 1;
      v[u] = A[(size_t)tc * n + mc];
      if (dal) v[u] *= dal[tc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = tb + u * dt;
      if (t < N) lcol[2 * pd_fpad(t)] = inb ? v[u] : 0.0;
    }
  }
  __syncthreads();
  fft_lds<double, false>(lds, N, C, stride, twl);

  // this thread's mode and frequencies k = t0 + u dt < N/2 (at most 8:
  // T >= C N / 8), plus k = N/2 for the threads tid < S
  const int half = N / 2;
  const Cx *ccol = lds + (pnt >> 1) * stride;
  const double m = mk[mc], kap = kk[mc];
  Cx X[9];
  double bs = 0.0, fs = 0.0;
  auto split = [&](int k) -> Cx {
    const Cx zk = ccol[pd_fpad(k)];
    const Cx zn = ccol[pd_fpad((N - k) & (N - 1))];
    return (pnt & 1) ? Cx{0.5 * (zk.im + zn.im), 0.5 * (zn.re - zk.re)}
                     : Cx{0.5 * (zk.re + zn.re), 0.5 * (zk.im - zn.im)};
  };
  // per frequency: omega^k = exp(-2 pi i k/N) from the LDS twiddle tables,
  // lambda_k = 1 - w omega^k, gamma_k = omega^k / N (times 2 for the
  // conjugate half, k = 1..N/2-1)
  const Cx *thi = twl + pd_tw_lo(N);
  const double invNd = 1.0 / (double)N;
  auto omega = [&](int k) -> Cx { return cmul(thi[k >> 6], twl[k & 63]); };
  auto recip = [](double x) {   // 1/x: hardware estimate and two Newton steps
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  };
  // 1 / (lambda_k m + kap)
  auto dinv = [&](Cx om) -> Cx {
    const Cx d = {(1.0 - w * om.re) * m + kap, -w * om.im * m};
    const double s2 = recip(d.re * d.re + d.im * d.im);
    return Cx{d.re * s2, -d.im * s2};
  };
  auto accumulate = [&](int k, Cx x) {
    const Cx om = omega(k);
    const Cx inv = dinv(om);
    const double g = ((k == 0 || k == half) ? 1.0 : 2.0) * invNd;
    const Cx L = {m * (x.re * inv.re - x.im * inv.im), m * (x.re * inv.im + x.im * inv.re)};
    bs += g * (om.re * L.re - om.im * L.im);
    fs += w * g * m * (om.re * inv.re - om.im * inv.im);
  };
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = t0 + u * dt;
    X[u] = split(k < half ? k : 0);
    if (k < half) accumulate(k, X[u]);
  }
  if (tid < S) {
    X[8] = split(half);
    accumulate(half, X[8]);
  }
  // sums over the threads of one mode: lanes l and l' share a mode when
  // l = l' mod S; then the waves, in order
  for (int off = 32; off >= S; off >>= 1) {
    bs += __shfl_xor(bs, off, 64);
    fs += __shfl_xor(fs, off, 64);
  }
  const int wid = tid >> 6, lane = tid & 63;
  if (lane < S) {
    sb[wid * S + lane] = bs;
    sf[wid * S + lane] = fs;
  }
  __syncthreads();
  double bt = 0.0, ft = 0.0;
  for (int q = 0; q < nw; ++q) {
    bt += sb[q * S + pnt];
    ft += sf[q * S + pnt];
  }
  const double x = bt / (1.0 + ft);
  // U~_k = m (X_k - w x) / d_k, then repack the two real columns
  auto solved = [&](int k, Cx v) -> Cx {
    const Cx inv = dinv(omega(k));
    const Cx r = {m * (v.re - w * x), m * v.im};
    return Cx{r.re * inv.re - r.im * inv.im, r.re * inv.im + r.im * inv.re};
  };
  Cx *wcol = lds + (pnt >> 1) * stride;
  auto pack = [&](int k, Cx mine) {
    const Cx other = {__shfl_xor(mine.re, 1, 64), __shfl_xor(mine.im, 1, 64)};
    Cx a = (pnt & 1) ? other : mine, b = (pnt & 1) ? mine : other;
    if (k == 0 || k == half) { a.im = 0.0; b.im = 0.0; }
    if (!(pnt & 1)) wcol[pd_fpad(k)] = Cx{a.re - b.im, a.im + b.re};
    else if (k > 0 && k < half) wcol[pd_fpad(N - k)] = Cx{a.re + b.im, b.re - a.im};
  };
  // every read of the spectrum above precedes the barrier
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = t0 + u * dt;
    const Cx y = solved(k < half ? k : 0, X[u]);
    if (k < half) pack(k, y);
  }
  if (tid < S) pack(half, solved(half, X[8]));
  __syncthreads();
  fft_lds<double, true>(lds, N, C, stride, twl);
  const double invN = 1.0 / (double)N;
  for (int tb = t0; tb < N; tb += 8 * dt) {
    double val[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = tb + u * dt;
      const int tc = t < N ? t : 0;
      const Cx z = ccol[pd_fpad(tc)];
      val[u] = ((pnt & 1) ? z.im : z.re) * invN;
      if (dalinv) val[u] *= dalinv[tc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = tb + u * dt;
      if (t < N && inb) B[(size_t)t * n + mode] = val[u];
    }
  }
}

}  // namespace

// Host side --------------------------------------------------------------

int pd_sine_dst_C(int n, int ell) {
  const int H = (n + 1) / 2;
  int C = 1;
  while (C < 32 && C * H < 4096 && 2 * C <= ell) C *= 2;
  return C;
}

size_t pd_sine_dst_lds(int n, int C) {
  const int H = (n + 1) / 2;
  const int T = C * H / 8;
  return ((size_t)C * pd_fft_col_stride(H) + pd_tw_entries(H)) * 16 + (size_t)T * 8;
}

size_t pd_sine_modal_lds(pd_plan p, int threads) {
  const int S = 2 * p->fft_C;
  return ((size_t)p->fft_C * p->fft_stride + pd_tw_entries(p->ell)) * 16 +
         2 * (size_t)(threads / 64) * S * 8;
}

pd_status pd_launch_sine_dst(pd_plan p, int mode, const double *u0, const double *F,
                             const double *in, double *out) {
  if (p->dst_L) return pd_launch_dst_rows1d(p, mode, u0, F, in, out);   // any n
  const int n = p->n, H = (n + 1) / 2, C = p->sine_C;
  const int T = C * H / 8;
  if (T < 1 || T > 512 || p->ell % C != 0) return PD_EINVAL;
  const int stride = pd_fft_col_stride(H);
  const size_t lds = pd_sine_dst_lds(n, C);
  auto twH = reinterpret_cast<const cpx<double> *>(p->sine_twH);
  auto wN = reinterpret_cast<const cpx<double> *>(p->sine_wN);
  if (mode == 0)
    hipLaunchKernelGGL(dst_rows_kernel<0>, dim3(p->ell / C), dim3(T), lds, p->stream, n, C,
                       stride, p->tau, u0, F, nullptr, p->sine_q, wN, twH, out);
  else
    hipLaunchKernelGGL(dst_rows_kernel<1>, dim3(p->ell / C), dim3(T), lds, p->stream, n, C,
                       stride, p->tau, nullptr, nullptr, in, p->sine_q, wN, twH, out);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_launch_sine_modal(pd_plan p, const double *A, double *B) {
  const int C = p->fft_C, N = p->ell;
  int need = C * N / 8;
  if (need < 64) need = 64;
  const int T = ((need + 63) / 64) * 64;
  if (T > 512) return PD_EINVAL;
  const int blocks = (p->n + 2 * C - 1) / (2 * C);
  const double *dal = p->alpha == 1.0 ? nullptr : p->dal;
  hipLaunchKernelGGL(sine_modal_kernel, dim3(blocks), dim3(T), pd_sine_modal_lds(p, T),
                     p->stream, N, p->n, C, p->fft_stride, A, dal,
                     reinterpret_cast<const cpx<double> *>(p->tw64), p->sine_m, p->sine_k, p->w,
                     B);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

void pd_sine_set_attributes(size_t max_lds) {
  const int v = (int)max_lds;
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_rows_kernel<0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_rows_kernel<1>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&sine_modal_kernel), v);
}
