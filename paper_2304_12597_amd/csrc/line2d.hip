// 2D shifted solves by separation (Section 6.1, 2D heat equation with
// K = I (x) T + T (x) I): after an orthonormal DST-I along x, the shifted
// block P_k = lambda_k I + tau K splits, for every x-sine-mode m with
// T s_m = theta_m s_m, into one tridiagonal system along y,
//
//     ((lambda_k + tau theta_m) I + tau T) y = d,
//
// so the parfor over k becomes a parfor over (k, m) of n-row line solves.
// Spectra here are [ell/2+1][n*n] in the DST-x domain, index y*n + m.  A block
// owns S consecutive m for one frequency (mode 1) or for a range of
// frequencies (modes 0 and 2, which sum over k); its tile [y][m0..m0+S) is
// staged through LDS with coalesced row segments, and each line is solved by
// P threads from constants precomputed per (k, m): float64 lines of at most
// one wave by the recurrence form of pd_scan.h (the lines are symmetric
// Toeplitz), the others by the chunked solver of pd_partition.h.
#include "pd_partition.h"
#include "pd_scan.h"

namespace {

template <typename R, int MR, int MODE, bool SCAN>
__global__ void __launch_bounds__(512, 4)
line2d_kernel(int n, int F2, int P, int S, int mgroups, int kchunk,
              const cpx<R> *__restrict__ fac, R toff, const double *__restrict__ gw,
              const cpx<R> *__restrict__ in, const double *__restrict__ vin,
              const double *__restrict__ xv, double wscale, cpx<R> *__restrict__ out,
              double *__restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int NF = 6 * (MR - 1);
  const int tid = threadIdx.x;
  const int g = tid / P;
  const int lt = tid - g * P;
  const int rows = P * MR;
  const int sstride = rows + 2;
  const size_t nbar = (size_t)n * n;
  cpx<R> *stage = reinterpret_cast<cpx<R> *>(smem_raw) + (size_t)g * sstride;
  Row3<R> *xch = reinterpret_cast<Row3<R> *>(smem_raw) + (size_t)g * P;
  size_t region = (size_t)S * sstride * sizeof(cpx<R>);
  const size_t accb = (size_t)S * rows * sizeof(double);
  if (accb > region) region = accb;
  region = (region + 15) & ~(size_t)15;
  cpx<R> *lfac_all = reinterpret_cast<cpx<R> *>(smem_raw + region);
  cpx<R> *lfac = lfac_all + (size_t)g * NF;

  const int mg = blockIdx.x % mgroups;
  const int m0 = mg * S;
  const int m = m0 + g;
  const bool mact = m < n;
  const int s0 = lt * MR;
  int len = n - s0;
  len = len < 0 ? 0 : (len > MR ? MR : len);
  int kbeg, kend;
  if (MODE == 1) {
    kbeg = blockIdx.x / mgroups;
    kend = kbeg + 1;
  } else {
    const int kc = blockIdx.x / mgroups;
    kbeg = kc * kchunk;
    kend = kbeg + kchunk < F2 ? kbeg + kchunk : F2;
  }
  const cpx<R> zero = {R(0), R(0)};
  const cpx<R> cc = {toff, R(0)};
  // tile entry idx = y S + gg (S a power of two): shifts, no division
  const int lgS = __builtin_ctz(S);
  const int tile = n * S;
  constexpr int U = 8;   // loads in flight per thread

  double acc[(MODE == 1) ? 1 : MR];
  R xr[(MODE == 2) ? 1 : MR];   // mode 1: -w x on this line; mode 2: v on this line
  R vr[(MODE == 2) ? MR : 1];
#pragma unroll
  for (int q = 0; q < MR; ++q) {
    if constexpr (MODE != 1) acc[q] = 0.0;
    const size_t i = (size_t)(s0 + q) * n + m;
    if constexpr (MODE == 1) xr[q] = (xv && mact && q < len) ? (R)(-wscale * xv[i]) : R(0);
    if constexpr (MODE == 2) vr[q] = (mact && q < len) ? (R)vin[i] : R(0);
  }

  for (int k = kbeg; k < kend; ++k) {
    __syncthreads();
    // (the recurrence form's table: its pd_scan_entries entries of each row)
    constexpr int NC = SCAN ? pd_scan_entries<MR>() : NF;
    for (int idx = tid; idx < S * NC; idx += blockDim.x) {
      const int gg = idx / NC, j = idx - gg * NC;
      const int mm = m0 + gg < n ? m0 + gg : n - 1;
      lfac_all[gg * NF + j] = fac[((size_t)k * n + mm) * NF + j];
    }
    if constexpr (MODE != 2) {
      // U loads in flight per thread (at clamped, valid addresses), then the
      // LDS stores; columns past n stage zeros
      const cpx<R> *src = in + (size_t)k * nbar;
      for (int b = tid; b < tile; b += U * (int)blockDim.x) {
        cpx<R> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = b + u * (int)blockDim.x;
          const int ic = idx < tile ? idx : tile - 1;
          const int y = ic >> lgS, mm = m0 + (ic & (S - 1));
          const cpx<R> t = src[(size_t)y * n + (mm < n ? mm : n - 1)];
          v[u] = pd_sel(mm < n, t, zero);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int idx = b + u * (int)blockDim.x;
          if (idx < tile)
            reinterpret_cast<cpx<R> *>(smem_raw)[(size_t)(idx & (S - 1)) * sstride + (idx >> lgS) + 1] = v[u];
        }
      }
    }
    __syncthreads();
    cpx<R> d[MR];
#pragma unroll
    for (int q = 0; q < MR; ++q) {
      cpx<R> v = zero;
      if (q < len) {
        if constexpr (MODE == 2) {
          v.re = vr[q];
        } else {
          v = stage[s0 + q + 1];
          if constexpr (MODE == 1) v.re += xr[q];
        }
      }
      d[q] = v;
    }
    if constexpr (SCAN)
      scan_solve_group<R, MR, CplxOps<R>, MODE == 1>(d, len, lt, P, lfac);
    else
      partition_solve<R, MR>(d, len, lt, P, lfac, xch, cc, cc);
    if constexpr (MODE == 1) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < MR; ++q)
        if (q < len) stage[s0 + q + 1] = d[q];
      __syncthreads();
      cpx<R> *dst = out + (size_t)k * nbar;
      for (int idx = tid; idx < tile; idx += blockDim.x) {
        const int y = idx >> lgS, gg = idx & (S - 1);
        const int mm = m0 + gg;
        if (mm < n)
          dst[(size_t)y * n + mm] =
              reinterpret_cast<cpx<R> *>(smem_raw)[(size_t)gg * sstride + y + 1];
      }
    } else {
      double gr = gw[2 * k], gi = gw[2 * k + 1];
      if constexpr (SCAN) {
        // the recurrence form returns kappa y: fold 1/kappa into the weight
        const cpx<R> ik = lfac[4];
        const double t = gr * (double)ik.re - gi * (double)ik.im;
        gi = gr * (double)ik.im + gi * (double)ik.re;
        gr = t;
      }
#pragma unroll
      for (int q = 0; q < MR; ++q)
        if (q < len) acc[q] += gr * (double)d[q].re - gi * (double)d[q].im;
    }
  }

  if constexpr (MODE != 1) {
    __syncthreads();
    double *sd = reinterpret_cast<double *>(smem_raw);
#pragma unroll
    for (int q = 0; q < MR; ++q) sd[(size_t)g * rows + s0 + q] = acc[q];
    __syncthreads();
    const int kc = blockIdx.x / mgroups;
    double *dst = partials + (size_t)kc * nbar;
    for (int idx = tid; idx < tile; idx += blockDim.x) {
      const int y = idx >> lgS, gg = idx & (S - 1);
      const int mm = m0 + gg;
      if (mm < n) dst[(size_t)y * n + mm] = sd[(size_t)gg * rows + y];
    }
  }
}

template <typename R, int MR, bool SCAN>
pd_status launch2d_form(pd_plan p, int mode, const void *in, const double *xv, void *out) {
  const Line2DConfig &L = p->l2d;
  const cpx<R> *fac = (sizeof(R) == 8) ? reinterpret_cast<const cpx<R> *>(p->fac64)
                                       : reinterpret_cast<const cpx<R> *>(p->fac32);
  const R toff = (R)p->uni[3];
  mode &= 0xff;
  if (mode == 1) {
    hipLaunchKernelGGL((line2d_kernel<R, MR, 1, SCAN>), dim3(p->F2 * L.mgroups), dim3(L.block),
                       L.lds, p->stream, p->n, p->F2, L.P, L.S, L.mgroups, L.kchunk, fac, toff,
                       p->gB64, reinterpret_cast<const cpx<R> *>(in), nullptr, xv, p->w,
                       reinterpret_cast<cpx<R> *>(out), nullptr);
  } else if (mode == 0) {
    hipLaunchKernelGGL((line2d_kernel<R, MR, 0, SCAN>), dim3(L.nkc * L.mgroups), dim3(L.block),
                       L.lds, p->stream, p->n, p->F2, L.P, L.S, L.mgroups, L.kchunk, fac, toff,
                       p->gB64, reinterpret_cast<const cpx<R> *>(in), nullptr, nullptr, p->w,
                       nullptr, p->partials);
  } else {
    hipLaunchKernelGGL((line2d_kernel<R, MR, 2, SCAN>), dim3(L.nkc * L.mgroups), dim3(L.block),
                       L.lds, p->stream, p->n, p->F2, L.P, L.S, L.mgroups, L.kchunk, fac, toff,
                       p->gJ64, nullptr, reinterpret_cast<const double *>(in), nullptr, p->w,
                       nullptr, p->partials);
  }
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

template <typename R, int MR>
pd_status launch2d(pd_plan p, int mode, const void *in, const double *xv, void *out) {
  if constexpr (sizeof(R) == 8) {
    if (pd_line2d_scan(p)) return launch2d_form<R, MR, true>(p, mode, in, xv, out);
  }
  return launch2d_form<R, MR, false>(p, mode, in, xv, out);
}

}  // namespace

Line2DConfig pd_choose_line2d(int n, int F2, int prec, int cus) {
  Line2DConfig L;
  const size_t cb = (prec == PD_FP64) ? 16 : 8;
  L.MR = (n <= 64) ? 4 : 8;
  L.P = 1;
  while (L.P * L.MR < n) L.P *= 2;
  L.S = 1;
  while (L.P * L.S * 2 <= 512) L.S *= 2;
  if (L.S > n) {
    L.S = 1;
    while (L.S * 2 <= n) L.S *= 2;
  }
  L.block = L.P * L.S;
  L.mgroups = (n + L.S - 1) / L.S;
  // enough blocks for the frequency sums: split k into chunks
  L.nkc = 1;
  while (L.nkc * L.mgroups < 2 * cus && L.nkc < F2) L.nkc *= 2;
  L.kchunk = (F2 + L.nkc - 1) / L.nkc;
  L.nkc = (F2 + L.kchunk - 1) / L.kchunk;
  const size_t rows = (size_t)L.P * L.MR;
  size_t region = (size_t)L.S * (rows + 2) * cb;
  const size_t accb = (size_t)L.S * rows * sizeof(double);
  if (accb > region) region = accb;
  region = (region + 15) & ~(size_t)15;
  L.lds = region + (size_t)L.S * 6 * (L.MR - 1) * cb;
  return L;
}

// Factors for every (k, m): b = lambda_k + tau theta_m + tau T_d, a = c = tau T_off.
void pd_line2d_factors(const pd_plan p, std::vector<double> &fac) {
  const int n = p->n, F2 = p->F2, MR = p->l2d.MR;
  const size_t NF = 6 * (size_t)(MR - 1);
  fac.assign((size_t)F2 * n * NF * 2, 0.0);
  const double tl = p->uni[3], td = p->uni[4];
  const bool scan = pd_line2d_scan(p);
  for (int k = 0; k < F2; ++k) {
    for (int m = 0; m < n; ++m) {
      const double theta = td + 2.0 * tl * std::cos((m + 1) * M_PI / (n + 1));
      if (scan) {
        // recurrence-form constants (pd_scan.h) at the same row stride
        pd_scan_table({tl, 0.0}, {p->lam[2 * k] + theta + td, p->lam[2 * k + 1]}, {tl, 0.0},
                      p->lam[2 * k + 1] == 0.0, n, MR,
                      reinterpret_cast<std::complex<double> *>(&fac[((size_t)k * n + m) * NF * 2]));
        continue;
      }
      pd_partition_factors(tl, 0.0, p->lam[2 * k] + theta + td, p->lam[2 * k + 1], tl, 0.0, MR,
                           &fac[((size_t)k * n + m) * NF * 2]);
    }
  }
}

pd_status pd_launch_line2d(pd_plan p, int mode, const void *in, const double *xv, void *out) {
  const int MR = p->l2d.MR;
  if (p->prec == PD_FP64) {
    if (MR == 4) return launch2d<double, 4>(p, mode, in, xv, out);
    if (MR == 8) return launch2d<double, 8>(p, mode, in, xv, out);
  } else {
    if (MR == 4) return launch2d<float, 4>(p, mode, in, xv, out);
    if (MR == 8) return launch2d<float, 8>(p, mode, in, xv, out);
  }
  pd_set_error("unsupported 2D line configuration");
  return PD_ENOTSUP;
}

void pd_line2d_set_attributes(size_t max_lds) {
  const int v = (int)max_lds;
  const void *fns[] = {
      reinterpret_cast<const void *>(&line2d_kernel<double, 4, 0, false>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 4, 0, true>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 4, 1, false>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 4, 1, true>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 4, 2, false>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 4, 2, true>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 8, 0, false>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 8, 0, true>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 8, 1, false>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 8, 1, true>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 8, 2, false>),
      reinterpret_cast<const void *>(&line2d_kernel<double, 8, 2, true>),
      reinterpret_cast<const void *>(&line2d_kernel<float, 4, 0, false>),
      reinterpret_cast<const void *>(&line2d_kernel<float, 4, 1, false>),
      reinterpret_cast<const void *>(&line2d_kernel<float, 4, 2, false>),
      reinterpret_cast<const void *>(&line2d_kernel<float, 8, 0, false>),
      reinterpret_cast<const void *>(&line2d_kernel<float, 8, 1, false>),
      reinterpret_cast<const void *>(&line2d_kernel<float, 8, 2, false>)};
  for (const void *f : fns)
    pd_set_max_lds(f, v);
}
