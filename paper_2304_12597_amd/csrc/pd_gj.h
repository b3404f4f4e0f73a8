// One-wave Gauss-Jordan inverse of a small shifted matrix, nu I + T (the
// per-frequency S_i of the projection methods for the capacitance system).
#pragma once
#include "pd_internal.h"

// One wave (a 64-thread block) inverts A = nu I + T (m x m, m <= MAXM <= 32;
// T real, row-major, leading dimension ldT) by Gauss-Jordan elimination with
// partial pivoting on the augmented matrix [A | I] in LDS: lane c owns column
// c of `a` (MAXM rows of 2 MAXM entries).  On return a[r][m + c] holds
// (A^{-1})_{r,c}.  The pivot of column col is the row r >= col with the
// largest |a[r][col]|^2, the first one on ties; fcol is MAXM entries of LDS.
template <int MAXM>
__device__ void wave_gj_inverse(int m, cpx<double> nu, const double *__restrict__ T, int ldT,
                                cpx<double> (*a)[2 * MAXM], cpx<double> *fcol) {
  using Cx = cpx<double>;
  const int lane = threadIdx.x;
  const int W = 2 * m;
  if (lane < W)
    for (int r = 0; r < m; ++r) {
      Cx v = {0.0, 0.0};
      if (lane < m) {
        v.re = T[(size_t)r * ldT + lane];
        if (r == lane) {
          v.re += nu.re;
          v.im += nu.im;
        }
      } else if (lane - m == r) {
        v.re = 1.0;
      }
      a[r][lane] = v;
    }
  __syncthreads();
  for (int col = 0; col < m; ++col) {
    double mag = -1.0;
    int idx = lane;
    if (lane >= col && lane < m) {
      const Cx v = a[lane][col];
      mag = v.re * v.re + v.im * v.im;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double om = __shfl_xor(mag, off, 64);
      const int oi = __shfl_xor(idx, off, 64);
      if (om > mag || (om == mag && oi < idx)) {
        mag = om;
        idx = oi;
      }
    }
    const int piv = idx;
    if (piv != col && lane < W) {
      const Cx t = a[col][lane];
      a[col][lane] = a[piv][lane];
      a[piv][lane] = t;
    }
    __syncthreads();
    const Cx inv = crecip(a[col][col]);
    __syncthreads();   // every lane has read the pivot
    if (lane < W) a[col][lane] = cmul(a[col][lane], inv);
    // column col of the other rows (unchanged by the scaling) before the
    // elimination overwrites it
    if (lane < m && lane != col) fcol[lane] = a[lane][col];
    __syncthreads();
    if (lane < W)
      for (int r = 0; r < m; ++r)
        if (r != col) a[r][lane] = csub(a[r][lane], cmul(fcol[r], a[col][lane]));
    __syncthreads();
  }
}
