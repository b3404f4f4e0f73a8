// Complex FFTs of C columns held in LDS (radix-8/4/2 Stockham autosort,
// in place), shared by the time transforms, the DST-I along x of the 2D path
// and the sine-basis transforms of the 1D path.  Column c, entry i sits at
// lds[c * stride + pd_fpad(i)]; twiddles come from two small LDS tables
// filled by tw_to_lds.  Forward: exp(-2 pi i jk/N); inverse: exp(+2 pi i
// jk/N), unscaled.
#pragma once
#include "pd_internal.h"

namespace pdfft {

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cpx<R> &x0, cpx<R> &x1, cpx<R> &x2, cpx<R> &x3) {
  cpx<R> s02 = cadd(x0, x2), d02 = csub(x0, x2);
  cpx<R> s13 = cadd(x1, x3), d13 = cmul_mi<R, INV>(csub(x1, x3));
  x0 = cadd(s02, s13);
  x2 = csub(s02, s13);
  x1 = cadd(d02, d13);
  x3 = csub(d02, d13);
}

template <typename R, bool INV>
__device__ __forceinline__ cpx<R> mul_w8(cpx<R> a) {
  // a * exp(-+ 2 pi i / 8)
  const R c = R(0.70710678118654752440084436210484904);
  return INV ? cpx<R>{c * (a.re - a.im), c * (a.re + a.im)}
             : cpx<R>{c * (a.re + a.im), c * (a.im - a.re)};
}

template <typename R, bool INV, int RAD>
__device__ __forceinline__ void small_dft(cpx<R> *v) {
  if constexpr (RAD == 2) {
    cpx<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (RAD == 4) {
    dft4<R, INV>(v[0], v[1], v[2], v[3]);
  } else {
    cpx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cpx<R> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<R, INV>(e0, e1, e2, e3);
    dft4<R, INV>(o0, o1, o2, o3);
    o1 = mul_w8<R, INV>(o1);
    o2 = cmul_mi<R, INV>(o2);
    o3 = cmul_mi<R, INV>(mul_w8<R, INV>(o3));
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
  }
}

// Copies the twiddle tables of a length-N transform (pd_tw_lo / pd_tw_entries)
// from the global table tw[m] = w^m into LDS; the caller synchronises.
template <typename R>
__device__ __forceinline__ void tw_to_lds(cpx<R> *lo, const cpx<R> *__restrict__ tw, int N) {
  const int LO = pd_tw_lo(N), E = pd_tw_entries(N);
  for (int m = threadIdx.x; m < E; m += blockDim.x) lo[m] = (m < LO) ? tw[m] : tw[(m - LO) * 64];
}

// x[r] *= w^r, r = 1..RAD-1, with the powers formed from w by products
template <typename R, int RAD>
__device__ __forceinline__ void twiddle_powers(cpx<R> *x, cpx<R> w1) {
  x[1] = cmul(x[1], w1);
  if constexpr (RAD >= 4) {
    const cpx<R> w2 = cmul(w1, w1), w3 = cmul(w2, w1);
    x[2] = cmul(x[2], w2);
    x[3] = cmul(x[3], w3);
    if constexpr (RAD == 8) {
      const cpx<R> w4 = cmul(w2, w2), w5 = cmul(w4, w1), w6 = cmul(w3, w3), w7 = cmul(w6, w1);
      x[4] = cmul(x[4], w4);
      x[5] = cmul(x[5], w5);
      x[6] = cmul(x[6], w6);
      x[7] = cmul(x[7], w7);
    }
  }
}

// One Stockham autosort stage of radix RAD over C columns of length N = 2^lgN
// held in LDS (entry i of column c at c * stride + pd_fpad(i)), in place: all
// reads, barrier, all writes.  Ns = 2^lgNs = length of the sub-transforms
// already done; the twiddles come from the LDS tables (lo, then hi).  Each
// thread handles up to 8/RAD butterflies (the host launches >= C*N/8
// threads).  All sizes are powers of two, so index arithmetic is shifts and
// masks; where the unpadded stride between a butterfly's RAD entries is a
// multiple of 8, the padded index is affine in the entry number.
template <typename R, bool INV, int RAD>
__device__ __forceinline__ void stockham_stage(cpx<R> *lds, int lgN, int lgNs, int C, int stride,
                                               const cpx<R> *lo) {
  constexpr int BPT = 8 / RAD;
  constexpr int LGR = RAD == 8 ? 3 : (RAD == 4 ? 2 : 1);
  const int T = blockDim.x, tid = threadIdx.x;
  const int N = 1 << lgN, Ns = 1 << lgNs;
  const int lgpc = lgN - LGR, per_col = 1 << lgpc;
  const int nb = C << lgpc;
  const int lgtw = lgN - lgNs - LGR;   // twiddle step N / (Ns * RAD)
  const cpx<R> *hi = lo + pd_tw_lo(N);
  const bool rlin = (per_col & 7) == 0;
  const int rstep = per_col + (per_col >> 3);
  const bool wlin = (Ns & 7) == 0 || (Ns == 1 && RAD == 8);
  const int wstep = Ns + (Ns >> 3);
  cpx<R> v[8];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * T;
    if (b < nb) {
      const int c = b >> lgpc, j = b & (per_col - 1);
      const cpx<R> *col = lds + c * stride;
      const int jm = j & (Ns - 1);
      if (rlin) {
        const cpx<R> *p = col + pd_fpad(j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[q * RAD + r] = p[r * rstep];
      } else {
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[q * RAD + r] = col[pd_fpad(j + r * per_col)];
      }
      if (Ns > 1) {
        const int m = jm << lgtw;
        cpx<R> w = cmul(hi[m >> 6], lo[m & 63]);
        if (INV) w.im = -w.im;
        twiddle_powers<R, RAD>(&v[q * RAD], w);
      }
      small_dft<R, INV, RAD>(&v[q * RAD]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * T;
    if (b < nb) {
      const int c = b >> lgpc, j = b & (per_col - 1);
      cpx<R> *col = lds + c * stride;
      const int jm = j & (Ns - 1);
      const int base = ((j >> lgNs) << (lgNs + LGR)) + jm;
      if (wlin) {
        cpx<R> *p = col + pd_fpad(base);
#pragma unroll
        for (int r = 0; r < RAD; ++r) p[r * wstep] = v[q * RAD + r];
      } else {
#pragma unroll
        for (int r = 0; r < RAD; ++r) col[pd_fpad(base + r * Ns)] = v[q * RAD + r];
      }
    }
  }
  __syncthreads();
}

template <typename R, bool INV>
__device__ __forceinline__ void fft_lds(cpx<R> *lds, int N, int C, int stride, const cpx<R> *twl) {
  const int lgN = __builtin_ctz(N);
  int lgNs = 0;
  while (lgNs + 3 <= lgN) {
    stockham_stage<R, INV, 8>(lds, lgN, lgNs, C, stride, twl);
    lgNs += 3;
  }
  if (lgNs + 2 == lgN) {
    stockham_stage<R, INV, 4>(lds, lgN, lgNs, C, stride, twl);
  } else if (lgNs + 1 == lgN) {
    stockham_stage<R, INV, 2>(lds, lgN, lgNs, C, stride, twl);
  }
}

}  // namespace pdfft
