// The capacitance product J_ell v = v + w sum_k gamma_k P_k^{-1} M v
// (eq. SMW_linearsystemII; eq. innersystem_alpha for alpha < 1) for 1D plans
// whose M and tau K are symmetric Toeplitz tridiagonals (uniform grids).
//
// The right-hand side M v is the same for every frequency, so the sum over
// frequencies is taken inside a chunked (partition) solve instead of after
// ell/2 + 1 separate ones.  The n rows are cut into nc <= 64 chunks of m rows
// (m odd; the last chunk L rows, 2 <= L <= m + 1).  With T_k the Toeplitz
// block of the first N = len - 1 rows of a chunk (sub- and super-diagonal
// a_k, diagonal b_k) and f_k = T_k^{-1} e_1 (T_k^{-1} e_N is f_k reversed,
// T_k being symmetric and persymmetric), the chunk's rows are
//
//   y_c[0..N) = T_k^{-1} r_c - a_k u_{k,c-1} f_k - a_k u_{k,c} rev(f_k),
//   y_c[N]    = u_{k,c}                      (the chunk's last unknown),
//
// with r = M v, and the chunks' last rows give a tridiagonal system in
// u_{k,0..nc-1} per frequency whose right-hand side needs E1 = f_k . r_c and
// E2 = rev(f_k) . r_c.  Summed over the frequencies with the weights
// g_k = w weight_k gamma_k (the conjugate half implied, real part):
//
//   (J v - v)_c[j] = (L r_c)[j]
//                    + Re sum_k zeta_k (f_k[j] u_{k,c-1} + f_k[N-1-j] u_{k,c}),
//   (J v - v)_c[N] = Re sum_k g_k u_{k,c},
//
// with zeta_k = -g_k a_k and L = S diag(rho) S, S the orthonormal DST-I of
// size N (it diagonalises every T_k), rho_i = Re sum_k g_k / (lambda_k m_i +
// tau kappa_i).  This reorders the same exact elimination.
//
// M is tridiag(ml, md, ml), so f . r_c = h . v_c + ml f[0] v[cm - 1]
// + ml f[N-1] v[cm + N] with h = M_N f: the dot products read v directly
// through the augmented vector [ml f[0], h, ml f[N-1]] over the window
// v[cm - 1 .. cm + N] (likewise L r_c with the rows of L M_N).
//
// Both contractions are dense and run on the fp64 matrix cores
// (v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; D row l / 16 + 4 r, column l % 16 sits in result r):
//
//   launch 1 (per 4 frequencies): E[4 freq x {E1, E2} x re/im][chunk] =
//     table[16 x window] . v-window[window x chunk] (v staged in LDS), the
//     last chunk's dots on the vector units, then the reduced system of each
//     frequency by parallel cyclic reduction across a wave -> U[k][c].
//   launch 2 (per 16-row tile x frequency split x block of column tiles):
//     out[row][chunk] = sum over the split's k and the 4 products
//     (re/im of u_{c-1}, u_c) of table[row][(k, p)] U[(k, p)][chunk], in
//     two halves of the split reduced in LDS; one more split holds L r_c.
//     The last chunk's rows and the chunks' last rows run on the vector
//     units, spread over the split's blocks.  Each split writes its own
//     partial tiles and rows (at most 16 n doubles in all).
//   launch 3: out = v + the splits' partials, added in split order.
//
// Frequency 0 (the smallest shift) stays out of the chunked sum when its
// shifted system is ill-conditioned: its term then comes from one block of
// the plan's shifted-solve kernel, the same rounded solve that passes B and C
// apply, so that the SMW reduction still cancels that rounding (pd_cp_tables).
//
// Every sum runs in a fixed order, so results do not depend on timing.
#include "pd_internal.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int CP1_WAVES = 5;                 // launch 1: 4 frequency slots + a paired real frequency
constexpr int CP1_BLOCK = 64 * CP1_WAVES;
constexpr int CP_SPLITS = 16;                // launch 2: frequency splits + the local term
constexpr int CP2_KW = 4;                    // launch 2: parts of a split per tile
constexpr int CP2_VW = 2;                    // launch 2: vector waves per block
constexpr int CP2_MAXW = 2 * CP2_KW + CP2_VW;   // launch 2: waves per block at most
constexpr int CP2_PF = 20;                   // launch 2: matrix-core steps loaded at once
constexpr int CP_UW = 66;                    // U row: zero, u_0 .. u_63, zero
constexpr int CP_PF = 36;                    // matrix-core steps whose operands are loaded at once

using Cx = cpx<double>;
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Cx shfl_c(Cx v, int src) {
  return Cx{__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}

// 1 / a for the reduced systems: the hardware reciprocal of |a|^2 refined by
// two Newton steps r <- r (2 - d r) (|a|^2 is far from the float64 range
// limits: the systems are diagonally dominant with entries of order one to
// tau kappa_max).
__device__ __forceinline__ Cx cp_recip(Cx a) {
  const double d = a.re * a.re + a.im * a.im;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return Cx{a.re * r, -a.im * r};
}

__device__ __forceinline__ v4d cp_mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Window index of step t for lane group gq (0..3) in a contraction of 4 Q
// window entries: blocks of 16 steps put the 4 groups 16 entries apart (so
// that 16 chunks at an odd stride and 4 groups read distinct LDS banks); a
// last partial block of R steps packs them R apart.  A bijection of
// {0..Q-1} x {0..3} onto {0..4Q-1}.
__host__ __device__ inline int cp_sidx(int t, int gq, int Q) {
  const int B16 = Q >> 4;
  if (t < (B16 << 4)) return ((t >> 4) << 6) + (gq << 4) + (t & 15);
  const int R = Q - (B16 << 4);
  return (B16 << 6) + R * gq + (t - (B16 << 4));
}

// v staged in LDS as vs[o + i] = v[i] (o = 2 for a 16-byte aligned v, else
// 1, so that the pairs v[2p + sh], v[2p + sh + 1] land on 16-byte LDS
// words, copied by direct 16-byte global -> LDS loads), zeros in [0, o) and
// [o + n, VL); returns o.  The caller waits (pd_wait_all) and syncs.
__device__ __forceinline__ int cp_stage_v(int n, int VL, const double *__restrict__ v, double *vs,
                                          int tid, int nthreads) {
  const int lane = tid & 63, wave = tid >> 6;
  const int sh = (int)((reinterpret_cast<uintptr_t>(v) >> 3) & 1);
  const int o = 2 - sh;
  const int np = (n - sh) >> 1;
  const double2 *src = reinterpret_cast<const double2 *>(v + sh);
  double2 *dst = reinterpret_cast<double2 *>(vs + 2);
  for (int p0 = wave * 64; p0 < np; p0 += nthreads)
    if (p0 + lane < np) pd_lds_dma16(src + p0 + lane, dst + p0);
  if (tid == 0) {
    if (sh) vs[o] = v[0];                              // the unpaired head
    if ((n - sh) & 1) vs[o + n - 1] = v[n - 1];        // the unpaired tail
  }
  if (tid < o) vs[tid] = 0.0;
  for (int j = o + n + tid; j < VL; j += nthreads) vs[j] = 0.0;
  return o;
}

// Window index of step t for lane group gq in the matrix-core contraction
// (see cp_sidx), written out for the device loops.
__device__ __forceinline__ int cp_sidx_d(int t, int gq, int B16, int R) {
  return t < (B16 << 4) ? ((t >> 4) << 6) + (gq << 4) + (t & 15)
                        : (B16 << 6) + R * gq + (t - (B16 << 4));
}

// acc += sum over the window (Q steps) of A . v-window for the 16 chunks of
// this wave's column tile: A for step t at At[t * 64] (lane-major), the
// window of chunk c at vc = vs + o - 1 + c m.  a0 holds the A operands of
// the first CP_PF steps (loaded by the caller ahead of the staging); later
// steps load CP_PF at a time.
__device__ __forceinline__ void cp_load_a(double (&a)[CP_PF], const double *__restrict__ At, int t0,
                                          int Q) {
#pragma unroll
  for (int u = 0; u < CP_PF; ++u) {
    const int t = t0 + u;
    a[u] = At[(t < Q ? t : Q - 1) * 64];
  }
}
__device__ __forceinline__ v4d cp_window_mfma(v4d acc, double (&a)[CP_PF],
                                              const double *__restrict__ At, const double *vc,
                                              int Q, int gq) {
  const int B16 = Q >> 4, R = Q & 15;
  for (int t0 = 0; t0 < Q; t0 += CP_PF) {
    if (t0 > 0) cp_load_a(a, At, t0, Q);
#pragma unroll
    for (int u0 = 0; u0 < CP_PF; u0 += 4) {
      double b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int t = t0 + u0 + u;
        t = t < Q ? t : Q - 1;
        b[u] = vc[cp_sidx_d(t, gq, B16, R)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (t0 + u0 + u < Q) acc = cp_mfma(a[u0 + u], b[u], acc);
    }
  }
  return acc;
}

// acc += sum over cnt steps of A_t B_t with lane operands A_t = pa[t * 64]
// and B_t = pb[t * sb] in global memory; the operands of up to PF steps are
// loaded at once.
template <int PF>
__device__ __forceinline__ v4d cp_global_mfma(v4d acc, const double *__restrict__ pa,
                                              const double *__restrict__ pb, long sb, int cnt) {
  for (int t0 = 0; t0 < cnt; t0 += PF) {
    double a[PF], b[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      int t = t0 + u;
      t = t < cnt ? t : cnt - 1;
      a[u] = pa[(long)t * 64];
      b[u] = pb[t * sb];
    }
#pragma unroll
    for (int u = 0; u < PF; ++u)
      if (t0 + u < cnt) acc = cp_mfma(a[u], b[u], acc);
  }
  return acc;
}

// Launch 1: the frequencies of slots 4 blockIdx.x .. + 3, wave q taking the
// reduced system of slot q's frequency.  With pair set, slot 0 of block 0
// holds the two real frequencies 0 and F2 - 1 (rows val 1 / 3 of the tile
// carry the second one's E1 / E2, whose imaginary parts vanish) and wave 4
// takes the reduced system of F2 - 1; then 4 gridDim.x + 1 = F2.  T1:
// [group][Q][64] matrix-core operands (row i = q + 4 val of the tile: val
// 0/1 = re/im of the augmented f, 2/3 = of its reverse); hL: [k][HLS]
// augmented last-chunk vectors; red: [k][8] reduced-system coefficients;
// U: [k][CP_UW] (column c + 1 = u_{k,c}).
__device__ __forceinline__ void cp_freq_body(const CpJob &J, const double *__restrict__ v,
                                             int blk) {
  const int n = J.n, F2 = J.F2, pair = J.pair, m = J.m, nc = J.nc, L = J.L, Q = J.Q;
  const int NTc = J.NTc, VL = J.VL, HLS = J.HLS;
  const double md = J.md, ml = J.ml;
  const double *__restrict__ T1 = J.T1;
  const Cx *__restrict__ hL = J.hL;
  const Cx *__restrict__ red = J.red;
  Cx *__restrict__ U = J.U;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *vs = reinterpret_cast<double *>(smem_raw);   // [VL]
  double *Ex = vs + VL;                                 // [CP1_WAVES][64][4]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gq = lane >> 4, cl = lane & 15;
  const int N0 = m - 1, NL = L - 1;
  const int Fs = pair ? F2 - 1 : F2;                    // frequencies in slots
  const bool paired = pair && blk == 0;
  // this wave's frequency (-1: none)
  const int kw = wave < 4 ? (4 * (int)blk + wave < Fs ? 4 * (int)blk + wave : -1)
                          : (paired ? F2 - 1 : -1);
  const int kq = kw >= 0 ? kw : 4 * (int)blk;
  const Cx zero = {0.0, 0.0};
  // reduced-system coefficients and the last chunk's first window entries of
  // this wave's frequency, loaded ahead of the staging
  const Cx *cf = red + (size_t)kq * 8;
  const bool lastlane = lane == nc - 1, pen = lane == nc - 2;
  const Cx ca = cf[0];
  const Cx clo = cf[lastlane ? 6 : 1];
  const Cx cdi = cf[lastlane ? 7 : (pen ? 4 : 2)];
  const Cx cup = cf[pen ? 5 : 3];
  const Cx *h = hL + (size_t)kq * HLS;
  const int s0 = lane < NL + 2 ? lane : NL + 1;
  const Cx h1a = h[s0], h2a = h[NL + 1 - s0];
  const int NT = NTc >> 4;
  const double *At = T1 + (size_t)blk * Q * 64 + lane;
  double a[CP_PF];
  if (wave < NT) cp_load_a(a, At, 0, Q);
  const int o = cp_stage_v(n, VL, v, vs, tid, CP1_BLOCK);
  pd_wait_all();
  __syncthreads();

  // ---- dot products of the interior chunks on the matrix cores ----
  if (wave < NT) {
    const int c = wave * 16 + cl;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    acc = cp_window_mfma(acc, a, At, vs + (o - 1) + c * m, Q, gq);
    if (c < nc - 1) {
      double *e = Ex + ((size_t)gq * 64 + c) * 4;
      if (paired && gq == 0) {
        double *e4 = Ex + ((size_t)4 * 64 + c) * 4;
        e[0] = acc[0];
        e[1] = 0.0;
        e[2] = acc[2];
        e[3] = 0.0;
        e4[0] = acc[1];
        e4[1] = 0.0;
        e4[2] = acc[3];
        e4[3] = 0.0;
      } else {
        e[0] = acc[0];
        e[1] = acc[1];
        e[2] = acc[2];
        e[3] = acc[3];
      }
    }
  }
  // ---- the last chunk's dots on the vector units: lanes = window ----
  if (kw >= 0) {
    const double *vl = vs + (o - 1) + (nc - 1) * m;
    Cx e1 = zero, e2 = zero;
    if (lane < NL + 2) {
      const double x = vl[lane];
      e1 = Cx{h1a.re * x, h1a.im * x};
      e2 = Cx{h2a.re * x, h2a.im * x};
    }
    for (int s = lane + 64; s < NL + 2; s += 64) {
      const double x = vl[s];
      const Cx h1 = h[s], h2 = h[NL + 1 - s];
      e1.re += h1.re * x;
      e1.im += h1.im * x;
      e2.re += h2.re * x;
      e2.im += h2.im * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
      e1.re += __shfl_xor(e1.re, off, 64);
      e1.im += __shfl_xor(e1.im, off, 64);
      e2.re += __shfl_xor(e2.re, off, 64);
      e2.im += __shfl_xor(e2.im, off, 64);
    }
    if (lane == 0) {
      double *e = Ex + ((size_t)wave * 64 + nc - 1) * 4;
      e[0] = e1.re;
      e[1] = e1.im;
      e[2] = e2.re;
      e[3] = e2.im;
    }
  }
  __syncthreads();

  // ---- the reduced system of this wave's frequency: lanes = chunks ----
  if (kw >= 0) {
    const int lc = lane < nc ? lane : nc - 1;
    const double *e = Ex + ((size_t)wave * 64 + lc) * 4;
    const Cx E1 = {e[0], e[1]}, E2 = {e[2], e[3]};
    // r = M v at the chunk's last row (row n - 1 for the last chunk)
    const int i = lc == nc - 1 ? n - 1 : lc * m + N0;
    const double rl = md * vs[o + i] + ml * (vs[o + i - 1] + vs[o + i + 1]);
    const Cx E1next = shfl_c(E1, lane + 1 < 64 ? lane + 1 : lane);
    Cx lo = zero, di = Cx{1.0, 0.0}, up = zero, rhs = zero;
    if (lane < nc) {
      lo = pd_sel(lane == 0, zero, clo);
      di = cdi;
      up = pd_sel(lastlane, zero, cup);
      Cx sum = E2;
      if (!lastlane) sum = cadd(sum, E1next);
      rhs = csub(Cx{rl, 0.0}, cmul(ca, sum));
    }
    const Cx rd = cp_recip(di);
    Cx al = cmul(lo, rd), ga = cmul(up, rd), de = cmul(rhs, rd);
    for (int st = 1; st < nc; st <<= 1) {
      const int sl = lane - st, sh = lane + st;
      const int slc = sl >= 0 ? sl : lane, shc = sh < 64 ? sh : lane;
      const Cx loa = pd_sel(sl >= 0, shfl_c(al, slc), zero);
      const Cx log_ = pd_sel(sl >= 0, shfl_c(ga, slc), zero);
      const Cx lod = pd_sel(sl >= 0, shfl_c(de, slc), zero);
      const Cx hia = pd_sel(sh < 64, shfl_c(al, shc), zero);
      const Cx hig = pd_sel(sh < 64, shfl_c(ga, shc), zero);
      const Cx hid = pd_sel(sh < 64, shfl_c(de, shc), zero);
      const Cx nb = csub(csub(Cx{1.0, 0.0}, cmul(al, log_)), cmul(ga, hia));
      const Cx nd = csub(csub(de, cmul(al, lod)), cmul(ga, hid));
      const Cx na = cneg(cmul(al, loa));
      const Cx ng = cneg(cmul(ga, hig));
      const Cx rb = cp_recip(nb);
      al = cmul(na, rb);
      ga = cmul(ng, rb);
      de = cmul(nd, rb);
    }
    // chunks past nc are zero
    Cx *row = U + (size_t)kw * CP_UW;
    row[1 + lane] = pd_sel(lane < nc, de, zero);
    if (lane < 2) row[lane == 0 ? 0 : CP_UW - 1] = zero;
  }
}

// Launch 2: block = (column-tile block nh, row tile mt, split sp).  Splits
// sp < Sk take frequencies [sp KPS, (sp + 1) KPS); split Sk (when local)
// takes L r_c.  Waves: (column tile, quarter of the split) for the matrix
// cores, the quarters added in LDS in a fixed order, then CP2_VW vector
// waves.  Outputs: the 16 x NTc tile of the split at tiles[(sp MT + mt)
// 16 NTc], and the split's vector rows vrow[sp NV + rho] (rho < NL: row rho
// of the last chunk; NL + c: the last row of chunk c), spread over the
// split's MT NH blocks (block b takes rho = b, b + MT NH, ...; lanes = 4
// rows x 16 frequency groups per wave).
__device__ __forceinline__ void cp_out_body(const CpJob &J, const double *__restrict__ v, int blk,
                                            int nthreads) {
  const int n = J.n, m = J.m, nc = J.nc, L = J.L, Q = J.Q, NTc = J.NTc, VL = J.VL, MT = J.MT;
  const int Sk = J.Sk, KPS = J.KPS, KPT = J.KPT, NH = J.NH;
  const double *__restrict__ T3 = J.T3;
  const Cx *__restrict__ c1 = J.c1;
  const Cx *__restrict__ gk = J.gk;
  const double *__restrict__ T4 = J.T4;
  const double *__restrict__ L1h = J.L1h;
  const Cx *__restrict__ U = J.U;
  double *__restrict__ tiles = J.tiles;
  double *__restrict__ vrow = J.vrow;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ v4d red2[(CP2_KW - 1) * 2 * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int gq = lane >> 4, cl = lane & 15;
  const int NL = L - 1;
  const int NT = NTc >> 4;
  const int TPB = NT / NH;                    // column tiles per block
  const int nh = blk % NH;
  const int mt = (blk / NH) % MT;
  const int sp = blk / (NH * MT);
  const int NV = NL + nc;
  double *tile = tiles + ((size_t)sp * MT + mt) * 16 * NTc;
  const int nmw = TPB * CP2_KW;                // matrix-core waves
  const double *Ud = reinterpret_cast<const double *>(U);
  double *vs = reinterpret_cast<double *>(smem_raw);
  int o = 0;
  if (sp >= Sk) {
    o = cp_stage_v(n, VL, v, vs, tid, nthreads);
    pd_wait_all();
    __syncthreads();
  }
  if (wave < nmw) {
    const int tl = wave % TPB, kh = wave / TPB;
    const int c = (nh * TPB + tl) * 16 + cl;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    if (sp < Sk) {
      const int qs = (KPS + CP2_KW - 1) / CP2_KW;
      const int kb = kh * qs < KPS ? kh * qs : KPS;
      const int ke = kb + qs < KPS ? kb + qs : KPS;
      const int ka = sp * KPS + kb;
      const double *pa = T3 + ((size_t)mt * KPT + ka) * 64 + lane;
      const double *pb = Ud + ((size_t)ka * CP_UW + c + (gq >> 1)) * 2 + (gq & 1);
      acc = cp_global_mfma<CP2_PF>(acc, pa, pb, 2L * CP_UW, ke - kb);
    } else if (kh == 0) {
      const double *At = T4 + (size_t)mt * Q * 64 + lane;
      double a[CP_PF];
      cp_load_a(a, At, 0, Q);
      acc = cp_window_mfma(acc, a, At, vs + (o - 1) + c * m, Q, gq);
    }
    // quarters of the split: the others add into the first in LDS (fixed order)
    if (kh > 0) red2[((kh - 1) * TPB + tl) * 64 + lane] = acc;
    __syncthreads();
    if (kh == 0) {
#pragma unroll
      for (int hh = 1; hh < CP2_KW; ++hh) {
        const v4d x = red2[((hh - 1) * TPB + tl) * 64 + lane];
        acc[0] += x[0];
        acc[1] += x[1];
        acc[2] += x[2];
        acc[3] += x[3];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) tile[(gq + 4 * r) * NTc + c] = acc[r];
    }
    return;
  }
  __syncthreads();   // the matrix-core waves' barrier
  // ---- the vector rows of this split: lanes = 4 rows x 16 frequency groups ----
  const int NB = MT * NH, b = mt * NH + nh;
  const int vw = wave - nmw;
  if (vw >= CP2_VW) return;   // a batched launch's waves beyond this problem's
  const int kg = lane & 15;
  constexpr int PFV = 8;
  for (int j0 = 0; b + j0 * NB < NV; j0 += 4 * CP2_VW) {
    const int rho = b + (j0 + 4 * vw + (lane >> 4)) * NB;
    const bool valid = rho < NV;
    double acc = 0.0;
    if (valid) {
      if (sp < Sk) {
        const int ka = sp * KPS;
        const int nit = (KPS - kg + 15) >> 4;    // k = ka + kg + 16 i, i < nit
        if (rho < NL) {
          const int s = rho;
          for (int i0 = 0; i0 < nit; i0 += PFV) {
            Cx a[PFV], bb[PFV], up[PFV], uc[PFV];
#pragma unroll
            for (int u = 0; u < PFV; ++u) {
              const int i = i0 + u < nit ? i0 + u : nit - 1;
              const size_t k = (size_t)ka + kg + 16 * i;
              a[u] = c1[k * NL + s];
              bb[u] = c1[k * NL + (NL - 1 - s)];
              up[u] = U[k * CP_UW + nc - 1];
              uc[u] = U[k * CP_UW + nc];
            }
#pragma unroll
            for (int u = 0; u < PFV; ++u)
              if (i0 + u < nit)
                acc += a[u].re * up[u].re - a[u].im * up[u].im + bb[u].re * uc[u].re -
                       bb[u].im * uc[u].im;
          }
        } else {
          const int cc = rho - NL;
          for (int i0 = 0; i0 < nit; i0 += PFV) {
            Cx g4[PFV], u4[PFV];
#pragma unroll
            for (int u = 0; u < PFV; ++u) {
              const int i = i0 + u < nit ? i0 + u : nit - 1;
              const size_t k = (size_t)ka + kg + 16 * i;
              g4[u] = gk[k];
              u4[u] = U[k * CP_UW + 1 + cc];
            }
#pragma unroll
            for (int u = 0; u < PFV; ++u)
              if (i0 + u < nit) acc += g4[u].re * u4[u].re - g4[u].im * u4[u].im;
          }
        }
      } else if (rho < NL) {
        const double *vl = vs + (o - 1) + (nc - 1) * m;
        const double *row = L1h + (size_t)rho * (NL + 2);
        for (int t = kg; t < NL + 2; t += 16) acc += row[t] * vl[t];
      }
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 8, 64);
    if (valid && kg == 0) vrow[(size_t)sp * NV + rho] = acc;
  }
}

// Launch 3: out = v + the splits' tiles and vector rows, summed in split
// order.  Items: MT x 16 x NTc tile entries, then the NV vector rows.
__device__ __forceinline__ void cp_sum_body(const CpJob &J, const double *__restrict__ v, int blk) {
  const int n = J.n, m = J.m, nc = J.nc, L = J.L, NTc = J.NTc, MT = J.MT, S = J.S;
  const double *__restrict__ tiles = J.tiles;
  const double *__restrict__ vrow = J.vrow;
  double *__restrict__ out = J.out;
  const int N0 = m - 1, NL = L - 1, NV = NL + nc;
  const int TS = 16 * NTc;
  const int nt = MT * TS;
  const int it = blk * 256 + threadIdx.x;
  if (it >= nt + NV) return;
  int i;
  const double *src;
  size_t stride;
  if (it < nt) {
    const int mt = it / TS, e = it - mt * TS, r = e / NTc, c = e - r * NTc;
    const int s = 16 * mt + r;
    if (c >= nc - 1 || s >= N0) return;
    i = c * m + s;
    src = tiles + it;
    stride = (size_t)MT * TS;
  } else {
    const int rho = it - nt;
    if (rho < NL) {
      i = (nc - 1) * m + rho;
    } else {
      const int c = rho - NL;
      i = c == nc - 1 ? n - 1 : c * m + N0;
    }
    src = vrow + rho;
    stride = (size_t)NV;
  }
  double y[CP_SPLITS];
#pragma unroll
  for (int q = 0; q < CP_SPLITS; ++q) y[q] = q < S ? src[q * stride] : 0.0;
  double s = v[i];
  if (J.extra) s += J.extra[i];
#pragma unroll
  for (int q = 0; q < CP_SPLITS; ++q) s += y[q];
  out[i] = s;
}


// The launches: one problem (the job by value), or a batch (jobs in device
// memory, block -> (job, local block) maps; the batched product of GMRES
// iteration jv reads v = job.v + jv n and skips problems that have stopped).
__global__ void __launch_bounds__(CP1_BLOCK) cp_freq_kernel(CpJob J) {
  if (J.skip && *J.skip != 0.0) return;
  cp_freq_body(J, J.v, blockIdx.x);
}
__global__ void __launch_bounds__(64 * CP2_MAXW) cp_out_kernel(CpJob J) {
  if (J.skip && *J.skip != 0.0) return;
  cp_out_body(J, J.v, blockIdx.x, blockDim.x);
}
__global__ void __launch_bounds__(256) cp_sum_kernel(CpJob J) {
  if (J.skip && *J.skip != 0.0) return;
  cp_sum_body(J, J.v, blockIdx.x);
}
__global__ void __launch_bounds__(CP1_BLOCK)
cp_freq_batch_kernel(const CpJob *__restrict__ jobs, const int2 *__restrict__ map,
                     const int *__restrict__ active, int jv) {
  const int2 e = map[blockIdx.x];
  if (active && !active[e.x]) return;
  const CpJob &J = jobs[e.x];
  if (J.skip && *J.skip != 0.0) return;
  cp_freq_body(J, J.v + (size_t)jv * J.n, e.y);
}
__global__ void __launch_bounds__(64 * CP2_MAXW)
cp_out_batch_kernel(const CpJob *__restrict__ jobs, const int2 *__restrict__ map,
                    const int *__restrict__ active, int jv) {
  const int2 e = map[blockIdx.x];
  if (active && !active[e.x]) return;
  const CpJob &J = jobs[e.x];
  if (J.skip && *J.skip != 0.0) return;
  cp_out_body(J, J.v + (size_t)jv * J.n, e.y, blockDim.x);
}
__global__ void __launch_bounds__(256)
cp_sum_batch_kernel(const CpJob *__restrict__ jobs, const int2 *__restrict__ map,
                    const int *__restrict__ active, int jv) {
  const int2 e = map[blockIdx.x];
  if (active && !active[e.x]) return;
  const CpJob &J = jobs[e.x];
  if (J.skip && *J.skip != 0.0) return;
  cp_sum_body(J, J.v + (size_t)jv * J.n, e.y);
}

void cis_pi(long k, long N, double &c, double &s) {
  // cos and sin of pi k / N with k reduced mod 2N first (exact argument)
  long r = k % (2 * N);
  if (r < 0) r += 2 * N;
  const double ang = M_PI * (double)r / (double)N;
  c = std::cos(ang);
  s = std::sin(ang);
}

struct HC { double re, im; };
inline HC hmul(HC a, HC b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline HC hadd(HC a, HC b) { return {a.re + b.re, a.im + b.im}; }
inline HC hsub(HC a, HC b) { return {a.re - b.re, a.im - b.im}; }
inline HC hscale(HC a, double s) { return {a.re * s, a.im * s}; }
inline HC hdiv(HC a, HC b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// f = T^{-1} e_1 for the symmetric Toeplitz tridiagonal tridiag(a, b, a) of
// size N (elimination without pivoting; T is diagonally dominant or an
// M-matrix times a shift with nonnegative real part).
void first_column(HC a, HC b, int N, HC *f) {
  std::vector<HC> cp(N), dp(N);
  cp[0] = hdiv(a, b);
  dp[0] = hdiv(HC{1.0, 0.0}, b);
  for (int i = 1; i < N; ++i) {
    const HC den = hsub(b, hmul(a, cp[i - 1]));
    cp[i] = hdiv(a, den);
    dp[i] = hdiv(HC{-(a.re * dp[i - 1].re - a.im * dp[i - 1].im),
                    -(a.re * dp[i - 1].im + a.im * dp[i - 1].re)}, den);
  }
  f[N - 1] = dp[N - 1];
  for (int i = N - 2; i >= 0; --i) f[i] = hsub(dp[i], hmul(cp[i], f[i + 1]));
}

// The augmented vector [ml f[0], (M_N f)[0..N), ml f[N-1]] (length N + 2).
void augment(const HC *f, int N, double md, double ml, HC *h) {
  h[0] = hscale(f[0], ml);
  for (int s = 0; s < N; ++s) {
    HC x = hscale(f[s], md);
    if (s > 0) x = hadd(x, hscale(f[s - 1], ml));
    if (s + 1 < N) x = hadd(x, hscale(f[s + 1], ml));
    h[s + 1] = x;
  }
  h[N + 1] = hscale(f[N - 1], ml);
}

// L = S diag(rho) S for the DST-I of size N, returned as the augmented rows
// of L M_N (N x (N + 2)); rho_i = Re sum_{k >= kfrom} g_k / (lam_k m_i + tau
// kappa_i).  False (and zeros) when every rho_i is zero.
bool local_matrix(pd_plan p, int N, int kfrom, std::vector<double> &Lh) {
  const int F2 = p->F2;
  const double ml = p->uni[0], md = p->uni[1], tkl = p->uni[3], tkd = p->uni[4];
  std::vector<double> rho(N), S((size_t)N * N);
  bool any = false;
  const double sc = std::sqrt(2.0 / (N + 1));
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double cc, ss;
      cis_pi((long)(i + 1) * (j + 1), N + 1, cc, ss);
      S[(size_t)i * N + j] = sc * ss;
    }
  for (int i = 0; i < N; ++i) {
    double cc, ss;
    cis_pi(i + 1, N + 1, cc, ss);
    const double mi = md + 2.0 * ml * cc, ki = tkd + 2.0 * tkl * cc;
    double s = 0.0;
    for (int k = kfrom; k < F2; ++k) {
      const HC d{p->lam[2 * k] * mi + ki, p->lam[2 * k + 1] * mi};
      s += hdiv(HC{p->gJ[2 * k], p->gJ[2 * k + 1]}, d).re;
    }
    rho[i] = s;
    any |= s != 0.0;
  }
  Lh.assign((size_t)N * (N + 2), 0.0);
  if (!any) return false;
  std::vector<double> Lm((size_t)N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int t = 0; t < N; ++t) {
      const double w = S[(size_t)i * N + t] * rho[t];
      for (int j = 0; j < N; ++j) Lm[(size_t)i * N + j] += w * S[(size_t)t * N + j];
    }
  for (int i = 0; i < N; ++i) {
    const double *row = &Lm[(size_t)i * N];
    double *h = &Lh[(size_t)i * (N + 2)];
    h[0] = ml * row[0];
    for (int s = 0; s < N; ++s) {
      double x = md * row[s];
      if (s > 0) x += ml * row[s - 1];
      if (s + 1 < N) x += ml * row[s + 1];
      h[s + 1] = x;
    }
    h[N + 1] = ml * row[N - 1];
  }
  return true;
}

}  // namespace

// Chunking of n rows: nc <= 64 chunks of m rows (m odd, at least 3), the
// last one L rows with 2 <= L <= m + 1.
void pd_cp_chunking(int n, int *m_out, int *nc_out, int *L_out) {
  int m = (n + 63) / 64;
  if (m < 3) m = 3;
  if (m % 2 == 0) ++m;
  int nc = (n + m - 1) / m;
  int L = n - (nc - 1) * m;
  if (L == 1 && nc > 1) {
    --nc;
    L = m + 1;
  }
  *m_out = m;
  *nc_out = nc;
  *L_out = L;
}

bool pd_cp_eligible(int n, int dims, int bdf_s, bool uniform, const double *uni) {
  return dims == 1 && bdf_s == 1 && uniform && n >= 2 && uni[0] == uni[2] && uni[3] == uni[5];
}

// Table and workspace sizes (doubles) and their offsets.
CpLayout pd_cp_layout(int n, int F2) {
  CpLayout c;
  pd_cp_chunking(n, &c.m, &c.nc, &c.L);
  c.N0 = c.m - 1;
  c.NL = c.L - 1;
  c.Q = (c.N0 + 2 + 3) / 4;
  c.NT = (c.nc + 15) / 16;
  c.NTc = 16 * c.NT;
  c.NH = c.NT % 2 == 0 ? c.NT / 2 : c.NT;   // blocks per row tile and split: 2 or 1 column tiles each
  // LDS index o + i of v[i] with o <= 2; windows reach o - 1 + (NTc - 1) m + 4 Q - 1
  const int vl = std::max(n + 3, (c.NTc - 1) * c.m + 4 * c.Q + 2);
  c.VL = (vl + 1) & ~1;
  c.G1 = (F2 + 3) / 4;
  c.G1run = c.G1;
  c.MT = (c.N0 + 15) / 16;
  c.Sk = CP_SPLITS - 1;
  c.KPS = (F2 + c.Sk - 1) / c.Sk;
  c.KPT = std::max(4 * c.G1, c.Sk * c.KPS);
  c.HLS = c.NL + 2;
  c.NV = c.NL + c.nc;
  size_t o = 0;
  auto take = [&o](size_t cnt) { const size_t at = o; o += (cnt + 1) & ~(size_t)1; return at; };
  c.T1 = take((size_t)c.G1 * c.Q * 64);
  c.hL = take(2 * (size_t)4 * c.G1 * c.HLS);
  c.red = take(16 * (size_t)F2);
  c.gk = take(2 * (size_t)c.KPT);
  c.T3 = take((size_t)c.MT * c.KPT * 64);
  c.c1 = take(2 * (size_t)c.KPT * c.NL);
  c.T4 = take((size_t)c.MT * c.Q * 64);
  c.L1h = take((size_t)c.NL * (c.NL + 2));
  c.gJ0 = take(2 * (size_t)F2);
  c.tables = o;
  c.U = take(2 * (size_t)c.KPT * CP_UW);
  c.tiles = take((size_t)CP_SPLITS * c.MT * 16 * c.NTc);
  c.vrow = take((size_t)CP_SPLITS * c.NV);
  c.total = o;
  return c;
}

// The tables of a plan (float64, host) and zeros for the workspace: lam, gJ
// and the uniform coefficients come from the plan.
void pd_cp_tables(pd_plan p, std::vector<double> &tab) {
  CpLayout &c = p->cpl;
  const int F2 = p->F2, N0 = c.N0, NL = c.NL, Q = c.Q;
  tab.assign(c.total, 0.0);
  const double ml = p->uni[0], md = p->uni[1], tkl = p->uni[3], tkd = p->uni[4];
  std::vector<HC> fa((size_t)N0), fb((size_t)NL), ha((size_t)N0 + 2), hb((size_t)NL + 2);
  auto put = [&tab](size_t at, HC z) {
    tab[at] = z.re;
    tab[at + 1] = z.im;
  };
  // Frequency 0 (the smallest shift, lam_0 = 1 - alpha^(1/ell)) leaves the
  // chunked sum when its shifted system is ill-conditioned enough to matter:
  // the passes apply a fixed rounded factorisation of P_0 everywhere, and the
  // SMW reduction cancels that perturbation only if the capacitance product
  // applies the same one.  Estimate of the inconsistency otherwise: |J - I|
  // on the smoothest sine mode x cond(P_0) x u; above 1e-12 the k = 0 term is
  // computed by the plan's shifted-solve kernel (one block) instead.
  {
    const int nn = p->n;
    double c1c, s1c, cnc, snc;
    cis_pi(1, nn + 1, c1c, s1c);
    cis_pi(nn, nn + 1, cnc, snc);
    const double m1 = md + 2.0 * ml * c1c, k1 = tkd + 2.0 * tkl * c1c;
    const double mn = md + 2.0 * ml * cnc, kn = tkd + 2.0 * tkl * cnc;
    double jm1 = 0.0;
    for (int k = 0; k < F2; ++k) {
      const HC d{p->lam[2 * k] * m1 + k1, p->lam[2 * k + 1] * m1};
      jm1 += hdiv(HC{p->gJ[2 * k] * m1, p->gJ[2 * k + 1] * m1}, d).re;
    }
    const double l0 = p->lam[0];
    const double e1 = std::fabs(l0 * m1 + k1), en = std::fabs(l0 * mn + kn);
    const double cond0 = std::max(e1, en) / std::max(std::min(e1, en), 1e-300);
    const double est = std::fabs(jm1) * cond0 * std::ldexp(1.0, -53);
    c.k0sep = est > 1e-12 ? 1 : 0;
    if (c.k0sep) {
      tab[c.gJ0] = p->gJ[0];
      tab[c.gJ0 + 1] = p->gJ[1];
    }
  }
  // the two real frequencies 0 and F2 - 1 (ell even) share slot 0 of the
  // first launch's block 0 when that makes the slots a multiple of 4
  const int last = F2 - 1;
  c.pair = p->ell % 2 == 0 && F2 >= 5 && last % 4 == 0 && p->lam[1] == 0.0 &&
           p->gJ[1] == 0.0 && p->lam[2 * last + 1] == 0.0 && p->gJ[2 * last + 1] == 0.0;
  c.G1run = c.pair ? last / 4 : c.G1;
  for (int k = 0; k < F2; ++k) {
    const HC lam{p->lam[2 * k], p->lam[2 * k + 1]};
    const HC g{p->gJ[2 * k], p->gJ[2 * k + 1]};
    const HC a{lam.re * ml + tkl, lam.im * ml};
    const HC b{lam.re * md + tkd, lam.im * md};
    first_column(a, b, N0, fa.data());
    first_column(a, b, NL, fb.data());
    augment(fa.data(), N0, md, ml, ha.data());
    augment(fb.data(), NL, md, ml, hb.data());
    const HC gc = (c.k0sep && k == 0) ? HC{0.0, 0.0} : g;   // weight in the chunked sum
    const HC zeta = hmul(HC{-gc.re, -gc.im}, a);
    // launch 1: matrix-core operands of group k / 4, tile row q + 4 val (the
    // paired real frequency F2 - 1: rows val 1 / 3 of slot 0 in group 0)
    const bool second = c.pair && k == last;
    const int grp = second ? 0 : k >> 2, q = second ? 0 : k & 3;
    for (int t = 0; t < Q; ++t)
      for (int l = 0; l < 64; ++l) {
        const int i = l & 15;
        if ((i & 3) != q) continue;
        const int val = i >> 2, s = cp_sidx(t, l >> 4, Q);
        if (s >= N0 + 2) continue;
        const HC h = val < 2 ? ha[s] : ha[N0 + 1 - s];
        if (second) {
          if (val & 1) tab[c.T1 + ((size_t)grp * Q + t) * 64 + l] = h.re;
        } else if (!(c.pair && k == 0 && (val & 1))) {
          tab[c.T1 + ((size_t)grp * Q + t) * 64 + l] = (val & 1) ? h.im : h.re;
        }
      }
    for (int s = 0; s < NL + 2; ++s) put(c.hL + 2 * ((size_t)k * c.HLS + s), hb[s]);
    put(c.gk + 2 * (size_t)k, gc);
    // launch 2: rows s of tile mt, products p = re/im of u_{c-1}, u_c
    for (int mt = 0; mt < c.MT; ++mt)
      for (int l = 0; l < 64; ++l) {
        const int s = 16 * mt + (l & 15), pp = l >> 4;
        if (s >= N0) continue;
        const HC z = hmul(zeta, fa[pp < 2 ? s : N0 - 1 - s]);
        tab[c.T3 + ((size_t)mt * c.KPT + k) * 64 + l] = (pp & 1) ? -z.im : z.re;
      }
    for (int s = 0; s < NL; ++s) put(c.c1 + 2 * ((size_t)k * NL + s), hmul(zeta, fb[s]));
    // reduced-system coefficients: a, lo/di/up of interior chunks, di/up of
    // the chunk before the last, lo/di of the last chunk
    const HC a2 = hmul(a, a);
    const HC lo_i = hmul(HC{-a2.re, -a2.im}, fa[N0 - 1]);
    const HC di_i = hsub(b, hmul(HC{2.0 * a2.re, 2.0 * a2.im}, fa[0]));
    const HC di_pen = hsub(hsub(b, hmul(a2, fa[0])), hmul(a2, fb[0]));
    const HC up_pen = hmul(HC{-a2.re, -a2.im}, fb[NL - 1]);
    const HC lo_L = hmul(HC{-a2.re, -a2.im}, fb[NL - 1]);
    const HC di_L = hsub(b, hmul(a2, fb[0]));
    const HC vals[8] = {a, lo_i, di_i, lo_i, di_pen, up_pen, lo_L, di_L};
    for (int w = 0; w < 8; ++w) put(c.red + 2 * ((size_t)k * 8 + w), vals[w]);
  }
  // the chunk-local term L r_c: zero exactly when every rho_i is zero in
  // float64 (long horizons: (1 + tau kappa_1 / m_1)^ell overflows the terms)
  std::vector<double> Lh0, Lh1;
  const bool l0 = local_matrix(p, N0, c.k0sep, Lh0);
  const bool l1 = local_matrix(p, NL, c.k0sep, Lh1);
  c.local = (l0 || l1) ? 1 : 0;
  for (int mt = 0; mt < c.MT; ++mt)
    for (int t = 0; t < Q; ++t)
      for (int l = 0; l < 64; ++l) {
        const int s = 16 * mt + (l & 15), w = cp_sidx(t, l >> 4, Q);
        if (s >= N0 || w >= N0 + 2) continue;
        tab[c.T4 + ((size_t)mt * Q + t) * 64 + l] = Lh0[(size_t)s * (N0 + 2) + w];
      }
  for (size_t i = 0; i < Lh1.size(); ++i) tab[c.L1h + i] = Lh1[i];
}

size_t pd_cp_lds1(const CpLayout &c) {
  return ((size_t)c.VL + CP1_WAVES * 64 * 4) * sizeof(double);
}
size_t pd_cp_lds2(const CpLayout &c) { return (size_t)c.VL * sizeof(double); }

// The product runs on these kernels when both launches' LDS fits (launch 2
// also holds (CP2_KW - 1) x 2 x 64 x 32 bytes of static LDS).
bool pd_cp_fits(int n, int F2, size_t max_lds) {
  const CpLayout c = pd_cp_layout(n, F2);
  return pd_cp_lds1(c) <= max_lds &&
         pd_cp_lds2(c) + (size_t)(CP2_KW - 1) * 2 * 64 * 32 <= max_lds;
}

void pd_cp_set_attributes(size_t max_lds) {
  const void *fns[] = {reinterpret_cast<const void *>(&cp_freq_kernel),
                       reinterpret_cast<const void *>(&cp_out_kernel),
                       reinterpret_cast<const void *>(&cp_freq_batch_kernel),
                       reinterpret_cast<const void *>(&cp_out_batch_kernel)};
  for (const void *fn : fns) pd_set_max_lds(fn, (int)max_lds);
}

CpJob pd_cp_job(pd_plan p, const double *v, double *Jv, const double *skip) {
  const CpLayout &c = p->cpl;
  double *t = p->cp_tab;
  CpJob J;
  J.n = p->n; J.F2 = p->F2; J.pair = c.pair; J.m = c.m; J.nc = c.nc; J.L = c.L; J.Q = c.Q;
  J.NTc = c.NTc; J.VL = c.VL; J.MT = c.MT; J.Sk = c.Sk; J.KPS = c.KPS; J.KPT = c.KPT;
  J.NH = c.NH; J.HLS = c.HLS; J.S = c.Sk + c.local;
  J.md = p->uni[1]; J.ml = p->uni[0];
  J.v = v; J.out = Jv; J.skip = skip;
  J.T1 = t + c.T1; J.T3 = t + c.T3; J.T4 = t + c.T4; J.L1h = t + c.L1h;
  J.hL = reinterpret_cast<const Cx *>(t + c.hL);
  J.red = reinterpret_cast<const Cx *>(t + c.red);
  J.c1 = reinterpret_cast<const Cx *>(t + c.c1);
  J.gk = reinterpret_cast<const Cx *>(t + c.gk);
  J.U = reinterpret_cast<Cx *>(t + c.U);
  J.tiles = t + c.tiles; J.vrow = t + c.vrow;
  J.extra = c.k0sep ? p->partials : nullptr;
  return J;
}

int pd_cp_blocks(const CpJob &J, int launch) {
  if (launch == 1) return J.pair ? (J.F2 - 1) / 4 : (J.F2 + 3) / 4;
  if (launch == 2) return J.MT * J.S * J.NH;
  const int items = J.MT * 16 * J.NTc + (J.L - 1) + J.nc;
  return (items + 255) / 256;
}

int pd_cp_threads2(const CpJob &J) { return 64 * ((J.NTc / 16 / J.NH) * CP2_KW + CP2_VW); }

size_t pd_cp_lds(const CpJob &J, int launch) {
  if (launch == 1) return ((size_t)J.VL + CP1_WAVES * 64 * 4) * sizeof(double);
  return J.S > J.Sk ? (size_t)J.VL * sizeof(double) : 0;
}

pd_status pd_cp_apply(pd_plan p, const double *v, double *Jv) {
  const CpJob J = pd_cp_job(p, v, Jv, p->gm_skip);
  if (p->cpl.k0sep) {
    const pd_status s0 = pd_launch_j_first_item(p, v, p->cp_tab + p->cpl.gJ0);
    if (s0 != PD_OK) return s0;
  }
  hipLaunchKernelGGL(cp_freq_kernel, dim3(pd_cp_blocks(J, 1)), dim3(CP1_BLOCK), pd_cp_lds(J, 1),
                     p->stream, J);
  PD_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(cp_out_kernel, dim3(pd_cp_blocks(J, 2)), dim3(pd_cp_threads2(J)),
                     pd_cp_lds(J, 2), p->stream, J);
  PD_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(cp_sum_kernel, dim3(pd_cp_blocks(J, 3)), dim3(256), 0, p->stream, J);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}

pd_status pd_cp_launch_batch(const CpJob *jobs, const int2 *map1, int nb1, const int2 *map2,
                             int nb2, int threads2, const int2 *map3, int nb3, size_t lds1,
                             size_t lds2, const int *active, int jv, hipStream_t s) {
  if (nb1 == 0) return PD_OK;
  hipLaunchKernelGGL(cp_freq_batch_kernel, dim3(nb1), dim3(CP1_BLOCK), lds1, s, jobs, map1,
                     active, jv);
  PD_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(cp_out_batch_kernel, dim3(nb2), dim3(threads2), lds2, s, jobs, map2, active,
                     jv);
  PD_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(cp_sum_batch_kernel, dim3(nb3), dim3(256), 0, s, jobs, map3, active, jv);
  PD_HIP_CHECK(hipGetLastError());
  return PD_OK;
}
