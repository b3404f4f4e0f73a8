// Time-axis DFTs of the space-time block (Section 2: post-multiplication by
// F^T diagonalises the circulant C_1; Section 4: with D_alpha scaling).
//
// The space-time arrays are time-major [ell][nbar] (float64), so the DFT runs
// along the strided axis.  One block owns a tile of 2*C consecutive spatial
// points over all ell time steps: global loads and stores touch 2*C
// consecutive doubles (or complex values) per time row, and the transform
// itself runs in LDS.  Two real columns are packed into one complex column
// (z = h_a + i h_b), transformed with a Stockham radix-8/4/2 FFT in LDS, and
// separated again with the conjugate symmetry of real transforms, so only
// the half spectrum k = 0..ell/2 is stored: frequency-major [ell/2+1][nbar].
#include "pd_internal.h"
#include "pd_residual.h"
#include "pd_fft.h"

namespace {

using namespace pdfft;

template <typename R, int MODE>
__device__ __forceinline__ void fft_forward_body(int tile, int N, int n, int nbar, int dims, int C,
                                                 int stride, double tau,
                                                 const double *__restrict__ u0,
                                                 const double *__restrict__ F,
                                                 const double *__restrict__ U,
                                                 const double *__restrict__ coef,
                                                 const double *__restrict__ dal,
                                                 const cpx<R> *__restrict__ tw,
                                                 cpx<R> *__restrict__ out,
                                                 double *__restrict__ red) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<R> *lds = reinterpret_cast<cpx<R> *>(smem_raw);
  cpx<R> *twl = lds + C * stride;
  tw_to_lds(twl, tw, N);
  const int T = blockDim.x, tid = threadIdx.x;
  const int lgS = __builtin_ctz(C) + 1, S = 2 * C;
  const int i0 = tile * S;
  // T is a multiple of S: every thread owns one point of the tile and the
  // time rows t0, t0 + dt, ... (entry t*S + pnt of the tile is thread
  // (t*S + pnt) mod T's)
  const int pnt = tid & (S - 1);
  const int t0 = tid >> lgS, dt = T >> lgS;
  const int i = i0 + pnt;
  const bool inb = i < nbar;
  const int ic = inb ? i : nbar - 1;
  R *lcol = reinterpret_cast<R *>(lds + (pnt >> 1) * stride) + (pnt & 1);
  double rn2 = 0.0, gn2 = 0.0;
  // Issue UNR independent loads per thread before storing to LDS, so their
  // HBM latencies overlap instead of adding up (16: a whole 2048-step column
  // pair of 512 threads in one round; the residual form, with more loads per
  // entry, 8): every load reads a clamped, valid address, and out-of-tile
  // entries are zeroed afterwards.  dal == NULL: alpha = 1, no scaling.
  constexpr int UNR = MODE == 1 ? 8 : 16;
  double h0 = 0.0;   // u0 at this point (used by the t = 0 entry)
  if (MODE == 0) h0 = u0[ic];
  for (int tb = t0; tb < N; tb += UNR * dt) {
    double vals[UNR];
    if constexpr (MODE != 1) {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int t = tb + u * dt;
        const int tc = t < N ? t : N - 1;
        vals[u] = F[(size_t)tc * nbar + ic];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int t = tb + u * dt;
        const int tc = t < N ? t : N - 1;
        double val = (MODE == 0) ? tau * vals[u] : vals[u];
        if (MODE == 0 && t == 0) val += h0;
        if (dal) val *= dal[tc];
        vals[u] = (t < N && inb) ? val : 0.0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int t = tb + u * dt;
        double val = 0.0;
        if (t < N && inb) {
          double r, g;
          residual_point(t, i, n, nbar, dims, tau, u0, F, U, coef, r, g);
          rn2 += r * r;
          gn2 += g * g;
          val = r;
          if (dal) val *= dal[t];
        }
        vals[u] = val;
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int t = tb + u * dt;
      if (t < N) lcol[2 * pd_fpad(t)] = (R)vals[u];
    }
  }
  __syncthreads();
  fft_lds<R, false>(lds, N, C, stride, twl);
  const int half = N / 2;
  // split the packed pairs: UNS outputs per thread per round, all LDS reads
  // before the stores (k < N/2 here, the Nyquist row k = N/2 below)
  const cpx<R> *ccol = lds + (pnt >> 1) * stride;
  constexpr int UNS = 8;
  for (int kb = t0; kb < half; kb += UNS * dt) {
    cpx<R> X[UNS];
#pragma unroll
    for (int u = 0; u < UNS; ++u) {
      const int k = kb + u * dt;
      const int kc = k < half ? k : 0;
      const cpx<R> zk = ccol[pd_fpad(kc)];
      const cpx<R> zn = ccol[pd_fpad((N - kc) & (N - 1))];
      const R xr = (pnt & 1) ? zk.im + zn.im : zk.re + zn.re;
      const R xi = (pnt & 1) ? zn.re - zk.re : zk.im - zn.im;
      X[u] = cpx<R>{R(0.5) * xr, R(0.5) * xi};
    }
#pragma unroll
    for (int u = 0; u < UNS; ++u) {
      const int k = kb + u * dt;
      if (k < half && inb) out[(size_t)k * nbar + i] = X[u];
    }
  }
  if (tid < S && inb) {
    const cpx<R> z = ccol[pd_fpad(half)];
    const R xr = (pnt & 1) ? z.im + z.im : z.re + z.re;
    const R xi = (pnt & 1) ? z.re - z.re : z.im - z.im;
    out[(size_t)half * nbar + i] = cpx<R>{R(0.5) * xr, R(0.5) * xi};
  }
  if (MODE == 1) {
    // block reduction of the two norms (float64)
    __shared__ double sr[32], sg[32];
    for (int off = 32; off > 0; off >>= 1) {
      rn2 += __shfl_down(rn2, off, 64);
      gn2 += __shfl_down(gn2, off, 64);
    }
    int wid = tid / 64, lane = tid % 64;
    __syncthreads();
    if (lane == 0) { sr[wid] = rn2; sg[wid] = gn2; }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < (T + 63) / 64; ++w) { a += sr[w]; b += sg[w]; }
      red[2 * tile] = a;
      red[2 * tile + 1] = b;
    }
  }
}

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Neighbouring tiles read the two halves of the same 128-byte lines, so map
// consecutive blocks of one XCD to consecutive tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  constexpr int X = 8;
  const int per = nb / X;            // tiles in the evenly divisible part
  if (b >= per * X) return b;        // remainder keeps its position
  return (b % X) * per + b / X;
}

template <typename R, int MODE>
__global__ void __launch_bounds__(1024)
fft_forward_kernel(int N, int n, int nbar, int dims, int C, int stride, double tau,
                   const double *__restrict__ u0, const double *__restrict__ F,
                   const double *__restrict__ U, const double *__restrict__ coef,
                   const double *__restrict__ dal, const cpx<R> *__restrict__ tw,
                   cpx<R> *__restrict__ out, double *__restrict__ red) {
  fft_forward_body<R, MODE>(xcd_tile(blockIdx.x, gridDim.x), N, n, nbar, dims, C, stride, tau,
                            u0, F, U, coef, dal, tw, out, red);
}

template <typename R, int ACC>
__device__ __forceinline__ void fft_inverse_body(int tile, int N, int nbar, int C, int stride,
                                                 const cpx<R> *__restrict__ in,
                                                 const double *__restrict__ dalinv,
                                                 const cpx<R> *__restrict__ tw,
                                                 double *__restrict__ U) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<R> *lds = reinterpret_cast<cpx<R> *>(smem_raw);
  cpx<R> *twl = lds + C * stride;
  tw_to_lds(twl, tw, N);
  const int T = blockDim.x, tid = threadIdx.x;
  const int lgC = __builtin_ctz(C), lgS = lgC + 1, S = 2 * C;
  const int i0 = tile * S;
  const int half = N / 2;
  constexpr int UNR = 8;
  // input: T is a multiple of C, so every thread owns one point pair c of
  // the tile and the frequencies k0, k0 + dk, ..., k <= N/2
  {
    const int c = tid & (C - 1);
    const int k0 = tid >> lgC, dk = T >> lgC;
    const int ia = i0 + 2 * c, ib = ia + 1;
    const int iac = ia < nbar ? ia : nbar - 1, ibc = ib < nbar ? ib : nbar - 1;
    cpx<R> *ccol = lds + c * stride;
    for (int kb = k0; kb <= half; kb += UNR * dk) {
      cpx<R> xa[UNR], xb[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        // clamped, valid addresses; out-of-tile values are zeroed after the loads
        const int k = kb + u * dk;
        const int kc = k <= half ? k : half;
        xa[u] = in[(size_t)kc * nbar + iac];
        xb[u] = in[(size_t)kc * nbar + ibc];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int k = kb + u * dk;
        const cpx<R> zc = {R(0), R(0)};
        xa[u] = pd_sel(k <= half && ia < nbar, xa[u], zc);
        xb[u] = pd_sel(k <= half && ib < nbar, xb[u], zc);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int k = kb + u * dk;
        if (k <= half) {
          cpx<R> a = xa[u], b = xb[u];
          if (k == 0 || k == half) { a.im = R(0); b.im = R(0); }
          ccol[pd_fpad(k)] = cpx<R>{a.re - b.im, a.im + b.re};
          if (k > 0 && k < half) ccol[pd_fpad(N - k)] = cpx<R>{a.re + b.im, b.re - a.im};
        }
      }
    }
  }
  __syncthreads();
  fft_lds<R, true>(lds, N, C, stride, twl);
  const double invN = 1.0 / (double)N;
  // output: every thread owns one point of the tile and the rows t0, t0 +
  // dt, ...; UNR2 outputs per round, the LDS reads and the dalinv (and,
  // accumulating, U) loads all issued before the stores
  constexpr int UNR2 = 8;
  const int pnt = tid & (S - 1);
  const int t0 = tid >> lgS, dt = T >> lgS;
  const int i = i0 + pnt;
  const bool inb = i < nbar;
  const int ic = inb ? i : nbar - 1;
  const cpx<R> *ocol = lds + (pnt >> 1) * stride;
  for (int tb = t0; tb < N; tb += UNR2 * dt) {
    double val[UNR2];
#pragma unroll
    for (int u = 0; u < UNR2; ++u) {
      const int t = tb + u * dt;
      const int tc = t < N ? t : 0;
      const cpx<R> z = ocol[pd_fpad(tc)];
      val[u] = (double)((pnt & 1) ? z.im : z.re) * invN;
      if (dalinv) val[u] *= dalinv[tc];
      if (ACC) val[u] += U[(size_t)tc * nbar + ic];
    }
#pragma unroll
    for (int u = 0; u < UNR2; ++u) {
      const int t = tb + u * dt;
      if (t < N && inb) U[(size_t)t * nbar + i] = val[u];
    }
  }
}

template <typename R, int ACC>
__global__ void __launch_bounds__(1024)
fft_inverse_kernel(int N, int nbar, int C, int stride, const cpx<R> *__restrict__ in,
                   const double *__restrict__ dalinv, const cpx<R> *__restrict__ tw,
                   double *__restrict__ U) {
  fft_inverse_body<R, ACC>(xcd_tile(blockIdx.x, gridDim.x), N, nbar, C, stride, in, dalinv, tw,
                           U);
}

// Orthonormal DST-I along x of every grid row (t, y) of a 2D space-time
// array [ell][n*n] (x fastest): S[m] = sqrt(2/(n+1)) sum_x v[x] sin((x+1)(m+1)
// pi/(n+1)).  It diagonalises the 1D factor T of K = I (x) T + T (x) I
// (Section 6.1) and is its own inverse.  Two rows share one complex FFT of
// length N = 2(n+1) of their odd extensions: with z = ext(a) + i ext(b),
// Z[k] = 2 S_b[k] - 2i S_a[k].
// MODE 0: v = h (tau f + u0 at t = 0); 1: v = float64 residual R (norms to
// red); 2: v = in.  ACC: out += S instead of out = S.
template <int MODE, int ACC>
__global__ void __launch_bounds__(1024)
dst_x_kernel(int n, int ell, int C, int stride, double tau, const double *__restrict__ u0,
             const double *__restrict__ F, const double *__restrict__ U,
             const double *__restrict__ in, const double *__restrict__ coef, Stencil2 sk,
             const cpx<double> *__restrict__ tw, double *__restrict__ out,
             double *__restrict__ red) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<double> *lds = reinterpret_cast<cpx<double> *>(smem_raw);
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 2 * (n + 1);
  const int nbar = n * n;
  const int rows = ell * n;
  const int r0 = blockIdx.x * 2 * C;
  cpx<double> *twl = lds + C * stride;
  tw_to_lds(twl, tw, N);
  double rn2 = 0.0, gn2 = 0.0;
  for (int c = tid; c < C; c += T) {
    lds[c * stride] = cpx<double>{0.0, 0.0};
    lds[c * stride + pd_fpad(n + 1)] = cpx<double>{0.0, 0.0};
  }
  constexpr int UNR = 8;
  // Elements are walked over rows padded to n + 1 (a power of two here), so
  // (row in block, x) come from shifts; the padding column is skipped.  The
  // block's first row gives (t0, y0) once; later rows step y with a carry.
  const int lgNP = __builtin_ctz(n + 1);
  const int total = (2 * C) << lgNP;
  const int t0 = r0 / n, y0 = r0 - t0 * n;
  auto row_ty = [&](int lr, int &t, int &y) {
    y = y0 + lr;
    t = t0;
    if (y >= n) {
      const int q = y / n;   // one step unless n < 2C
      t += q;
      y -= q * n;
    }
  };
  for (int base = tid; base < total; base += UNR * T) {
    double vals[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      double v = 0.0;
      const int lr = idx >> lgNP, x = idx & n;
      if (idx < total && x < n) {
        const int row = r0 + lr;
        if (row < rows) {
          int t, y;
          row_ty(lr, t, y);
          const int i = y * n + x;
          if (MODE == 0) {
            v = tau * F[(size_t)t * nbar + i];
            if (t == 0) v += u0[i];
          } else if (MODE == 1) {
            double r, g;
            residual_point_2d(t, x, y, n, nbar, tau, u0, F, U, coef, sk, r, g);
            rn2 += r * r;
            gn2 += g * g;
            v = r;
          } else {
            v = in[(size_t)t * nbar + i];
          }
        }
      }
      vals[u] = v;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      const int lr = idx >> lgNP, x = idx & n;
      if (idx < total && x < n) {
        double *p1 = reinterpret_cast<double *>(&lds[(lr >> 1) * stride + pd_fpad(x + 1)]);
        double *p2 = reinterpret_cast<double *>(&lds[(lr >> 1) * stride + pd_fpad(N - 1 - x)]);
        p1[lr & 1] = vals[u];
        p2[lr & 1] = -vals[u];
      }
    }
  }
  __syncthreads();
  fft_lds<double, false>(lds, N, C, stride, twl);
  const double scale = 0.5 * sqrt(2.0 / (double)(n + 1));
  // UNR outputs per thread per round, all reads before the stores
  for (int base = tid; base < total; base += UNR * T) {
    double s[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      const int ic = idx < total ? idx : 0;
      const int lr = ic >> lgNP, m0 = ic & n, m = m0 < n ? m0 : n - 1;
      const cpx<double> z = lds[(lr >> 1) * stride + pd_fpad(m + 1)];
      s[u] = ((lr & 1) ? z.re : -z.im) * scale;
      if (ACC) {
        int t, y;
        row_ty(r0 + lr < rows ? lr : rows - 1 - r0, t, y);
        s[u] += out[(size_t)t * nbar + (size_t)y * n + m];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      const int lr = idx >> lgNP, m = idx & n;
      if (idx < total && m < n) {
        const int row = r0 + lr;
        if (row < rows) {
          int t, y;
          row_ty(lr, t, y);
          out[(size_t)t * nbar + (size_t)y * n + m] = s[u];
        }
      }
    }
  }
  if (MODE == 1) {
    __shared__ double sr[32], sg[32];
    for (int off = 32; off > 0; off >>= 1) {
      rn2 += __shfl_down(rn2, off, 64);
      gn2 += __shfl_down(gn2, off, 64);
    }
    int wid = tid / 64, lane = tid % 64;
    __syncthreads();
    if (lane == 0) { sr[wid] = rn2; sg[wid] = gn2; }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < (T + 63) / 64; ++w) { a += sr[w]; b += sg[w]; }
      red[2 * blockIdx.x] = a;
      red[2 * blockIdx.x + 1] = b;
    }
  }
}

struct FftLaunch {
  int C, stride, threads, blocks;
  size_t lds;
};

FftLaunch fft_config(pd_plan p) {
  FftLaunch L;
  const int N = p->ell;
  const size_t cb = (p->prec == PD_FP64) ? 16 : 8;
  L.C = p->fft_C;
  L.stride = p->fft_stride;
  L.lds = ((size_t)L.C * L.stride + pd_tw_entries(N)) * cb;
  int need = L.C * N / 8;
  if (need < 64) need = 64;
  L.threads = ((need + 63) / 64) * 64;
  L.blocks = (p->nbar + 2 * L.C - 1) / (2 * L.C);
  return L;
}

}  // namespace

// Choose C (point pairs per block): keep LDS at <= 64 KiB where possible
// (two blocks per CU), else up to two point pairs per block; at most 512
// threads (C*N/8), and the tile no wider than the problem.
int pd_choose_fft_C(int ell, int nbar, int prec, size_t max_lds) {
  const size_t cb = (prec == PD_FP64) ? 16 : 8;
  const size_t col = (size_t)pd_fft_col_stride(ell) * cb, twb = pd_tw_entries(ell) * cb;
  int C = 1;
  while (C < 32 && 2 * C * col + twb <= 65536 && 2 * C * ell / 8 <= 512) C *= 2;
  while (C < 2 && 2 * C * col + twb <= max_lds && 2 * C * ell / 8 <= 512) C *= 2;
  int maxC = 1;
  while (2 * maxC < nbar && maxC < 32) maxC *= 2;
  if (C > maxC) C = maxC;
  return C;
}

// The transform bodies index with shifts: C must be a power of two <= 32
// (then the block size, a multiple of 64, is a multiple of 2C).
static bool fft_C_valid(int C) { return C >= 1 && C <= 32 && (C & (C - 1)) == 0; }

pd_status pd_launch_fft_forward(pd_plan p, const double *u0, const double *F,
                                const double *U, void *out, int mode) {
  FftLaunch L = fft_config(p);
  if (!fft_C_valid(L.C)) return PD_EINVAL;
  const double *dal = p->alpha == 1.0 ? nullptr : p->dal;   // D_alpha = I for alpha = 1
#define PD_FWD(R, M, TW, O)                                                                 \
  hipLaunchKernelGGL((fft_forward_kernel<R, M>), dim3(L.blocks), dim3(L.threads), L.lds,    \
                     p->stream, p->ell, p->n, p->nbar, p->dims, L.C, L.stride, p->tau, u0, \
                     F, U, p->coef64, dal, TW, O, p->red)
  if (p->prec == PD_FP64) {
    auto tw = reinterpret_cast<const cpx<double> *>(p->tw64);
    auto o = reinterpret_cast<cpx<double> *>(out);
    if (mode == 0) PD_FWD(double, 0, tw, o);
    else if (mode == 2) PD_FWD(double, 2, tw, o);
    else PD_FWD(double, 1, tw, o);
  } else {
    auto tw = reinterpret_cast<const cpx<float> *>(p->tw32);
    auto o = reinterpret_cast<cpx<float> *>(out);
    if (mode == 0) PD_FWD(float, 0, tw, o);
    else if (mode == 2) PD_FWD(float, 2, tw, o);
    else PD_FWD(float, 1, tw, o);
  }
#undef PD_FWD
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

namespace {

// Orthonormal DST-I along x for n + 1 not a power of two (chirp-z form).
// With j = x + 1, k = m + 1 and N1 = n + 1, jk = (j^2 + k^2 - (k - j)^2) / 2
// turns the sine sum into a convolution:
//   S[m] = sqrt(2/N1) Im(c_k sum_j (v_j c_j) conj(c_{k-j})),
//   c_j = exp(i pi j^2 / (2 N1)),
// a linear convolution of two length-n sequences, computed as a circular
// one of length L >= 2n - 1: FFT in LDS, times bhat (the transform of the
// wrapped conj(c_d), |d| < n, with 1/L folded in), inverse FFT.  One row
// per LDS column; MODE and ACC as for dst_x_kernel.  D1: the rows are the
// ell time rows of a 1D array [ell][n] (MODE 0 or 2) instead of the grid rows
// (t, y) of [ell][n*n].
template <int MODE, int ACC, bool D1 = false>
__global__ void __launch_bounds__(1024)
dst_x_chirp_kernel(int n, int ell, int Lc, int C, int stride, double tau,
                   const double *__restrict__ u0, const double *__restrict__ F,
                   const double *__restrict__ U, const double *__restrict__ in,
                   const double *__restrict__ coef, Stencil2 sk,
                   const cpx<double> *__restrict__ tw,
                   const cpx<double> *__restrict__ chirp, const cpx<double> *__restrict__ bhat,
                   double *__restrict__ out, double *__restrict__ red) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using Cx = cpx<double>;
  static_assert(!(D1 && MODE == 1), "1D rows: MODE 0 or 2");
  Cx *lds = reinterpret_cast<Cx *>(smem_raw);
  const int T = blockDim.x, tid = threadIdx.x;
  const int nbar = D1 ? n : n * n;
  const int rows = D1 ? ell : ell * n;
  const int r0 = blockIdx.x * C;
  const int lgL = __builtin_ctz(Lc);
  Cx *twl = lds + C * stride;
  tw_to_lds(twl, tw, Lc);
  double rn2 = 0.0, gn2 = 0.0;
  // entries n .. L-1 of every column are zero
  const int padn = Lc - n;
  for (int idx = tid; idx < C * padn; idx += T) {
    const int c = idx / padn, q = n + (idx - c * padn);
    lds[c * stride + pd_fpad(q)] = Cx{0.0, 0.0};
  }
  constexpr int UNR = 8;
  const int total = C * n;
  for (int base = tid; base < total; base += UNR * T) {
    double vals[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      double v = 0.0;
      if (idx < total) {
        const int lr = idx / n, x = idx - lr * n;
        const int row = r0 + lr;
        if (row < rows) {
          const int t = D1 ? row : row / n, y = D1 ? 0 : row - t * n;
          const int i = y * n + x;
          if (MODE == 0) {
            v = tau * F[(size_t)t * nbar + i];
            if (t == 0) v += u0[i];
          } else if (MODE == 1) {
            double r, g;
            residual_point_2d(t, x, y, n, nbar, tau, u0, F, U, coef, sk, r, g);
            rn2 += r * r;
            gn2 += g * g;
            v = r;
          } else {
            v = in[(size_t)t * nbar + i];
          }
        }
      }
      vals[u] = v;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      if (idx < total) {
        const int lr = idx / n, x = idx - lr * n;
        const Cx cj = chirp[x + 1];
        lds[lr * stride + pd_fpad(x)] = Cx{vals[u] * cj.re, vals[u] * cj.im};
      }
    }
  }
  __syncthreads();
  fft_lds<double, false>(lds, Lc, C, stride, twl);
  for (int idx = tid; idx < (C << lgL); idx += T) {
    const int c = idx >> lgL, q = idx & (Lc - 1);
    Cx *e = &lds[c * stride + pd_fpad(q)];
    *e = cmul(*e, bhat[q]);
  }
  __syncthreads();
  fft_lds<double, true>(lds, Lc, C, stride, twl);
  const double scale = sqrt(2.0 / (double)(n + 1));
  for (int base = tid; base < total; base += UNR * T) {
    double s[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      const int ic = idx < total ? idx : 0;
      const int lr = ic / n, m = ic - lr * n;
      const Cx z = lds[lr * stride + pd_fpad(m)];
      const Cx ck = chirp[m + 1];
      s[u] = (ck.re * z.im + ck.im * z.re) * scale;
      if (ACC) {
        int row = r0 + lr;
        row = row < rows ? row : rows - 1;
        const int t = D1 ? row : row / n, y = D1 ? 0 : row - t * n;
        s[u] += out[(size_t)t * nbar + (size_t)y * n + m];
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int idx = base + u * T;
      if (idx < total) {
        const int lr = idx / n, m = idx - lr * n;
        const int row = r0 + lr;
        if (row < rows) {
          const int t = D1 ? row : row / n, y = D1 ? 0 : row - t * n;
          out[(size_t)t * nbar + (size_t)y * n + m] = s[u];
        }
      }
    }
  }
  if (MODE == 1) {
    __shared__ double sr[32], sg[32];
    for (int off = 32; off > 0; off >>= 1) {
      rn2 += __shfl_down(rn2, off, 64);
      gn2 += __shfl_down(gn2, off, 64);
    }
    int wid = tid / 64, lane = tid % 64;
    __syncthreads();
    if (lane == 0) { sr[wid] = rn2; sg[wid] = gn2; }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < (T + 63) / 64; ++w) { a += sr[w]; b += sg[w]; }
      red[2 * blockIdx.x] = a;
      red[2 * blockIdx.x + 1] = b;
    }
  }
}
}  // namespace

namespace {
struct DstLaunch {
  int C, stride, threads, blocks;
  size_t lds;
};
// rows per block: 2C (pairs of rows per FFT column), C for the chirp-z form
DstLaunch dst_config(pd_plan p, int trows) {
  DstLaunch L;
  const int N = p->dst_L ? p->dst_L : 2 * (p->n + 1);
  L.C = p->dst_C;
  L.stride = pd_fft_col_stride(N);
  L.lds = ((size_t)L.C * L.stride + pd_tw_entries(N)) * 16;
  int need = L.C * N / 8;
  if (need < 64) need = 64;
  L.threads = ((need + 63) / 64) * 64;
  const int rows = trows * p->n;
  const int per = p->dst_L ? L.C : 2 * L.C;
  L.blocks = (rows + per - 1) / per;
  return L;
}
}  // namespace

// FFT length of the chirp-z DST-I of length n: 0 when n + 1 is a power of
// two (one FFT of length 2(n+1) per pair of rows), else the least power of
// two >= 2n - 1.
int pd_dst_chirp_length(int n) {
  if (((n + 1) & n) == 0) return 0;
  int L = 4;
  while (L < 2 * n - 1) L *= 2;
  return L;
}

int pd_choose_dst_C(int n) {
  const int Lc = pd_dst_chirp_length(n);
  const int N = Lc ? Lc : 2 * (n + 1);
  int C = 1;
  const size_t col = (size_t)pd_fft_col_stride(N) * 16, twb = pd_tw_entries(N) * 16;
  while (C < 16 && 2 * C * col + twb <= 65536 && 2 * C * N / 8 <= 1024) C *= 2;
  return C;
}

int pd_dst_blocks(pd_plan p) { return dst_config(p, p->ell).blocks; }

// tau T's constant diagonals for the residual stencil on uniform grids
static Stencil2 pd_stencil2(pd_plan p) {
  Stencil2 s;
  s.uni = p->uniform ? 1 : 0;
  s.kl = p->uni[3];
  s.kd = p->uni[4];
  s.ku = p->uni[5];
  return s;
}

pd_status pd_launch_dst_x(pd_plan p, int mode, const double *u0, const double *F,
                          const double *U, const double *in, double *out, int accumulate) {
  DstLaunch L = dst_config(p, p->ell);
  auto tw = reinterpret_cast<const cpx<double> *>(p->twd);
  if (p->dst_L) {
    auto ch = reinterpret_cast<const cpx<double> *>(p->twd + p->twd_chirp);
    auto bh = reinterpret_cast<const cpx<double> *>(p->twd + p->twd_bhat);
#define PD_DSTC(M, A)                                                                        \
  hipLaunchKernelGGL((dst_x_chirp_kernel<M, A>), dim3(L.blocks), dim3(L.threads), L.lds,     \
                     p->stream, p->n, p->ell, p->dst_L, L.C, L.stride, p->tau, u0, F, U, in,  \
                     p->coef64, pd_stencil2(p), tw, ch, bh, out, p->red)
    if (mode == 0) PD_DSTC(0, 0);
    else if (mode == 1) PD_DSTC(1, 0);
    else if (accumulate) PD_DSTC(2, 1);
    else PD_DSTC(2, 0);
#undef PD_DSTC
    PD_HIP_CHECK(hipGetLastError());
    return PD_OK;
  }
#define PD_DST(M, A)                                                                        \
  hipLaunchKernelGGL((dst_x_kernel<M, A>), dim3(L.blocks), dim3(L.threads), L.lds, p->stream, \
                     p->n, p->ell, L.C, L.stride, p->tau, u0, F, U, in, p->coef64,            \
                     pd_stencil2(p), tw, out, p->red)
  if (mode == 0) PD_DST(0, 0);
  else if (mode == 1) PD_DST(1, 0);
  else if (accumulate) PD_DST(2, 1);
  else PD_DST(2, 0);
#undef PD_DST
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// Orthonormal DST-I along x of `trows` time rows of `in` into `out` (or
// added to it): the mode-2 transform on a [trows][nbar] array.
pd_status pd_launch_dst_x_rows(pd_plan p, const double *in, double *out, int trows,
                               int accumulate) {
  DstLaunch L = dst_config(p, trows);
  auto tw = reinterpret_cast<const cpx<double> *>(p->twd);
  if (p->dst_L) {
    auto ch = reinterpret_cast<const cpx<double> *>(p->twd + p->twd_chirp);
    auto bh = reinterpret_cast<const cpx<double> *>(p->twd + p->twd_bhat);
    if (accumulate)
      hipLaunchKernelGGL((dst_x_chirp_kernel<2, 1>), dim3(L.blocks), dim3(L.threads), L.lds,
                         p->stream, p->n, trows, p->dst_L, L.C, L.stride, p->tau, nullptr,
                         nullptr, nullptr, in, p->coef64, pd_stencil2(p), tw, ch, bh, out, p->red);
    else
      hipLaunchKernelGGL((dst_x_chirp_kernel<2, 0>), dim3(L.blocks), dim3(L.threads), L.lds,
                         p->stream, p->n, trows, p->dst_L, L.C, L.stride, p->tau, nullptr,
                         nullptr, nullptr, in, p->coef64, pd_stencil2(p), tw, ch, bh, out, p->red);
    PD_HIP_CHECK(hipGetLastError());
    return PD_OK;
  }
  if (accumulate)
    hipLaunchKernelGGL((dst_x_kernel<2, 1>), dim3(L.blocks), dim3(L.threads), L.lds, p->stream,
                       p->n, trows, L.C, L.stride, p->tau, nullptr, nullptr, nullptr, in,
                       p->coef64, pd_stencil2(p), tw, out, p->red);
  else
    hipLaunchKernelGGL((dst_x_kernel<2, 0>), dim3(L.blocks), dim3(L.threads), L.lds, p->stream,
                       p->n, trows, L.C, L.stride, p->tau, nullptr, nullptr, nullptr, in,
                       p->coef64, pd_stencil2(p), tw, out, p->red);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

// Orthonormal DST-I of the ell time rows of a 1D array [ell][n] in chirp-z
// form (sine-basis plans with n + 1 not a power of two).  mode 0: rows
// h_t = tau f_t (+ u0 at t = 0); mode 1: rows of `in`.  out may equal in
// (a block reads its rows completely before it writes them).
pd_status pd_launch_dst_rows1d(pd_plan p, int mode, const double *u0, const double *F,
                               const double *in, double *out) {
  if (!p->dst_L) return PD_EINVAL;
  const int N = p->dst_L, C = p->dst_C;
  const int stride = pd_fft_col_stride(N);
  const size_t lds = ((size_t)C * stride + pd_tw_entries(N)) * 16;
  int need = C * N / 8;
  if (need < 64) need = 64;
  const int threads = ((need + 63) / 64) * 64;
  const int blocks = (p->ell + C - 1) / C;
  auto tw = reinterpret_cast<const cpx<double> *>(p->twd);
  auto ch = reinterpret_cast<const cpx<double> *>(p->twd + p->twd_chirp);
  auto bh = reinterpret_cast<const cpx<double> *>(p->twd + p->twd_bhat);
  if (mode == 0)
    hipLaunchKernelGGL((dst_x_chirp_kernel<0, 0, true>), dim3(blocks), dim3(threads), lds,
                       p->stream, p->n, p->ell, N, C, stride, p->tau, u0, F, nullptr, nullptr,
                       p->coef64, pd_stencil2(p), tw, ch, bh, out, p->red);
  else
    hipLaunchKernelGGL((dst_x_chirp_kernel<2, 0, true>), dim3(blocks), dim3(threads), lds,
                       p->stream, p->n, p->ell, N, C, stride, p->tau, nullptr, nullptr, nullptr,
                       in, p->coef64, pd_stencil2(p), tw, ch, bh, out, p->red);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_launch_fft_inverse(pd_plan p, const void *in, double *U, int accumulate) {
  FftLaunch L = fft_config(p);
  if (!fft_C_valid(L.C)) return PD_EINVAL;
  const double *dalinv = p->alpha == 1.0 ? nullptr : p->dal + p->ell;
#define PD_INV(R, A, TW, I)                                                                 \
  hipLaunchKernelGGL((fft_inverse_kernel<R, A>), dim3(L.blocks), dim3(L.threads), L.lds,    \
                     p->stream, p->ell, p->nbar, L.C, L.stride, I, dalinv, TW, U)
  if (p->prec == PD_FP64) {
    auto tw = reinterpret_cast<const cpx<double> *>(p->tw64);
    auto i = reinterpret_cast<const cpx<double> *>(in);
    if (accumulate) PD_INV(double, 1, tw, i);
    else PD_INV(double, 0, tw, i);
  } else {
    auto tw = reinterpret_cast<const cpx<float> *>(p->tw32);
    auto i = reinterpret_cast<const cpx<float> *>(in);
    if (accumulate) PD_INV(float, 1, tw, i);
    else PD_INV(float, 0, tw, i);
  }
#undef PD_INV
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

int pd_fft_blocks(pd_plan p) { return fft_config(p).blocks; }

// Allow the transform kernels the device's full LDS per block.
void pd_fft_set_attributes(size_t max_lds) {
  const int v = (int)max_lds;
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_forward_kernel<double, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_forward_kernel<double, 1>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_forward_kernel<float, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_forward_kernel<float, 1>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_forward_kernel<double, 2>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_forward_kernel<float, 2>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_kernel<0, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_kernel<1, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_kernel<2, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_kernel<2, 1>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_chirp_kernel<0, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_chirp_kernel<1, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_chirp_kernel<2, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_chirp_kernel<2, 1>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_chirp_kernel<0, 0, true>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&dst_x_chirp_kernel<2, 0, true>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_inverse_kernel<double, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_inverse_kernel<double, 1>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_inverse_kernel<float, 0>), v);
  pd_set_max_lds(reinterpret_cast<const void *>(&fft_inverse_kernel<float, 1>), v);
}

namespace {
template <typename R, int MODE>
__global__ void __launch_bounds__(1024)
fft_forward_batch_kernel(const FftJob *__restrict__ jobs, const int2 *__restrict__ map) {
  const int2 m = map[blockIdx.x];
  const FftJob &j = jobs[m.x];
  fft_forward_body<R, MODE>(m.y, j.N, j.n, j.nbar, j.dims, j.C, j.stride, j.tau, j.u0, j.F, j.U,
                            j.coef, j.dal, reinterpret_cast<const cpx<R> *>(j.tw),
                            reinterpret_cast<cpx<R> *>(j.spec), j.red);
}
template <typename R>
__global__ void __launch_bounds__(1024)
fft_inverse_batch_kernel(const FftJob *__restrict__ jobs, const int2 *__restrict__ map) {
  const int2 m = map[blockIdx.x];
  const FftJob &j = jobs[m.x];
  fft_inverse_body<R, 0>(m.y, j.N, j.nbar, j.C, j.stride,
                         reinterpret_cast<const cpx<R> *>(j.spec), j.dal ? j.dal + j.N : nullptr,
                         reinterpret_cast<const cpx<R> *>(j.tw), j.out);
}
}  // namespace

pd_status pd_launch_fft_forward_batch(int prec, const FftJob *jobs, const int2 *map, int nblocks,
                                      int threads, size_t lds, hipStream_t s) {
  if (nblocks == 0) return PD_OK;
  if (prec == PD_FP64)
    hipLaunchKernelGGL((fft_forward_batch_kernel<double, 0>), dim3(nblocks), dim3(threads), lds,
                       s, jobs, map);
  else
    hipLaunchKernelGGL((fft_forward_batch_kernel<float, 0>), dim3(nblocks), dim3(threads), lds,
                       s, jobs, map);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_launch_fft_inverse_batch(int prec, const FftJob *jobs, const int2 *map, int nblocks,
                                      int threads, size_t lds, hipStream_t s) {
  if (nblocks == 0) return PD_OK;
  if (prec == PD_FP64)
    hipLaunchKernelGGL((fft_inverse_batch_kernel<double>), dim3(nblocks), dim3(threads), lds, s,
                       jobs, map);
  else
    hipLaunchKernelGGL((fft_inverse_batch_kernel<float>), dim3(nblocks), dim3(threads), lds, s,
                       jobs, map);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

void pd_fft_batch_set_attributes(size_t max_lds) {
  const int v = (int)max_lds;
  const void *fns[] = {reinterpret_cast<const void *>(&fft_forward_batch_kernel<double, 0>),
                       reinterpret_cast<const void *>(&fft_forward_batch_kernel<float, 0>),
                       reinterpret_cast<const void *>(&fft_inverse_batch_kernel<double>),
                       reinterpret_cast<const void *>(&fft_inverse_batch_kernel<float>)};
  for (const void *fn : fns)
    pd_set_max_lds(fn, v);
}
