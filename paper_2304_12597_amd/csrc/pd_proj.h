// Projections of frequency-domain vectors onto a real orthonormal basis, the
// V_m^T h_i step of the projection methods for the capacitance system.
#pragma once
#include "pd_internal.h"

// A 256-thread block computes, for PT consecutive frequencies i0.. and PK
// consecutive basis vectors k0.., the sums sum_row V[k][row] h_i[row] with
// h_i = spec + i * n (rows strided over the threads: coalesced loads of V
// and h, each V value used PT times and each h value PK times).  Frequencies
// >= F2 and basis vectors >= nk contribute zeros.  On return thread
// t < PK * PT holds the sum for k = k0 + t / PT, i = i0 + t % PT in `out`.
constexpr int PROJ_PT = 4;
constexpr int PROJ_PK = 8;

__device__ inline void proj_tile(int n, int F2, int nk, const double *__restrict__ V,
                                 const cpx<double> *__restrict__ spec, int i0, int k0,
                                 cpx<double> &out) {
  constexpr int PT = PROJ_PT, PK = PROJ_PK;
  __shared__ double red[4][PK * PT][2];
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  double ar[PK][PT], ai[PK][PT];
#pragma unroll
  for (int kk = 0; kk < PK; ++kk)
#pragma unroll
    for (int f = 0; f < PT; ++f) {
      ar[kk][f] = 0.0;
      ai[kk][f] = 0.0;
    }
  for (int row = tid; row < n; row += 256) {
    cpx<double> hv[PT];
#pragma unroll
    for (int f = 0; f < PT; ++f)
      hv[f] = (i0 + f < F2) ? spec[(size_t)(i0 + f) * n + row] : cpx<double>{0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < PK; ++kk) {
      const double vk = (k0 + kk < nk) ? V[(size_t)(k0 + kk) * n + row] : 0.0;
#pragma unroll
      for (int f = 0; f < PT; ++f) {
        ar[kk][f] += vk * hv[f].re;
        ai[kk][f] += vk * hv[f].im;
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < PK; ++kk)
#pragma unroll
    for (int f = 0; f < PT; ++f) {
      double a = ar[kk][f], b = ai[kk][f];
      for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
      }
      if (lane == 0) {
        red[wid][kk * PT + f][0] = a;
        red[wid][kk * PT + f][1] = b;
      }
    }
  __syncthreads();
  if (tid < PK * PT) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 4; ++w) {
      a += red[w][tid][0];
      b += red[w][tid][1];
    }
    out = cpx<double>{a, b};
  }
}
