// Shifted solves of symmetric Toeplitz tridiagonal systems by two first-order
// recurrences: the parfor of shifted solves of Algorithm 1 (Section 2,
// P_k = lambda_k M + tau K) on uniform grids, passes B and C, and the 2D
// line solves after the DST along x (Section 6.1).
//
// For one frequency the system has constant sub-diagonal a, diagonal b and
// super-diagonal c.  Let kappa be the root of larger modulus of
// kappa^2 - b kappa + a c = 0, r1 = -a/kappa, r2 = -c/kappa, rho = r1 r2 and
// Z the down-shift.  Then kappa (1 + rho) = b and
//
//     P = kappa (I - r1 Z)(I - r2 Z^T) + kappa rho e_0 e_0^T,
//
// since the product of the two bidiagonal factors reproduces every row of P
// except the first, where it lacks rho x_0.  With
// S(y) = (I - r2 Z^T)^{-1} (I - r1 Z)^{-1} y -- a forward recurrence
// v_i = y_i + r1 v_{i-1} (v_{-1} = 0) and a backward one
// z_i = v_i + r2 z_{i+1} (z_n = 0) -- and w = S(e_0), the Sherman-Morrison
// formula for the corner term gives
//
//     x = (z - beta z_0 w) / kappa,   beta = rho / (1 + rho w_0).
//
// For P symmetric (a = c) r1 = r2 = r with |r| <= 1, so both recurrences
// are stable.  The corner term needs no second vector: z_0 = sum_i r^i v_i
// is a weighted sum of the forward values, so beta z_0 is known before the
// backward recurrence runs, and subtracting beta z_0 r^i from v_i (the
// forward recurrence of e_0 is r^i) makes the backward recurrence return
// kappa x directly.
//
// A group of P threads solves one system of n <= P*MR rows: thread lt owns
// rows [lt*MR, lt*MR + len), s0 = lt*MR.  The forward recurrence runs over
// the thread's rows from a zero start (u_q); the chunk carries are combined
// by a scan across the group that composes the chunk maps x -> R x + e
// (R = r^MR): DPP row shifts and row broadcasts inside a wave (lane shuffles
// of width P for groups smaller than a wave), then the waves' totals
// through LDS.  With ex = v at row s0-1, the chunk's rows are v_q = u_q + r^(q+1) ex,
// so its share of z_0 is r^s0 (sum_q r^q u_q + ex sum_{q<len} r^(2q+1)), and
// the corrected rows are u_q + r^q (r ex - beta z_0 r^s0): one pass over the
// rows after z_0 is summed.  The backward recurrence runs the same way.  No
// division and three block barriers per solve, against the log2(P)
// dependent reduction steps of a partition method.  The chunk start
// r^s0 = R^lt comes out of the forward scan (lane l ends with R^(l+1)).
//
// Per-frequency table (complex entries, built on the host by
// pd_scan_table; the kernels stage each system's row into LDS):
//   0 r1,  1 r2,  2 R1 = r1^MR,  3 R2 = r2^MR,  4 1/kappa,  5 beta,
//   6 sum_{q<MR} r^(2q+1),  7 + q: r^q for q = 0..MR (the symmetric r),
//   8 + MR: sum_{q < n mod MR} r^(2q+1) (the one ragged chunk's share).
// The powers of r inside a chunk come from the table, not from products.
#pragma once
#include <complex>
#include "pd_partition.h"

template <int MR>
constexpr int pd_scan_entries() { return 9 + MR; }

// Lane moves by DPP (data-parallel primitives: a VALU operand modifier, no
// LDS round trip).  CTRL: row_shr:s = 0x110 + s, row_shl:s = 0x100 + s,
// wave_shr:1 = 0x138, wave_shl:1 = 0x130, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.  Lanes whose source is outside the pattern, or whose
// row is off in ROWMASK, take `old`.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double pd_dpp(double v, double old) {
#if defined(__HIP_DEVICE_COMPILE__)
  const long long vb = __builtin_bit_cast(long long, v), ob = __builtin_bit_cast(long long, old);
  const int lo = __builtin_amdgcn_update_dpp((int)ob, (int)vb, CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(ob >> 32), (int)(vb >> 32), CTRL, ROWMASK, 0xF,
                                             false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
#else
  return v;
#endif
}
template <int CTRL, int ROWMASK, typename R>
__device__ __forceinline__ cpx<R> pd_dpp(cpx<R> v, cpx<R> old) {
  return cpx<R>{pd_dpp<CTRL, ROWMASK>(v.re, old.re), pd_dpp<CTRL, ROWMASK>(v.im, old.im)};
}
template <typename R>
__device__ __forceinline__ cpx<R> pd_readlane(cpx<R> v, int l) {
#if defined(__HIP_DEVICE_COMPILE__)
  auto rl = [l](double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
  };
  return cpx<R>{rl(v.re), rl(v.im)};
#else
  return v;
#endif
}

// One step of the inclusive scan of chunk maps (m, c) across a wave: lanes
// combine with the partial map of the lanes before them (identity: m = 1,
// c = 0, which `old` supplies where the pattern has no source).
template <int CTRL, int ROWMASK, typename A, typename R>
__device__ __forceinline__ void pd_scan_step(cpx<R> &c, cpx<R> &m) {
  const cpx<R> oc = pd_dpp<CTRL, ROWMASK>(c, cpx<R>{R(0), R(0)});
  const cpx<R> om = pd_dpp<CTRL, ROWMASK>(m, A::one());
  c = A::fma(c, m, oc);
  m = A::mul(m, om);
}

struct PdNoPrefetch {
  __device__ void operator()(int) const {}
};


// OPS as for partition_solve: CplxOps (one complex system) or DualOps (two
// real systems in the real and imaginary parts).  xw: 3*(P/64) complex LDS
// entries for the group.  LB: LDS-only barriers.  SCALE: return x; otherwise
// kappa x (the caller folds 1/kappa into its weights).  The group's P threads
// are whole waves (P a multiple of 64, P <= 512).  Every thread of the block
// calls this together; rows past the end of the system (q >= len) hold zero
// on entry and are left undefined.
template <typename R, int MR, typename A, bool LB, bool SCALE, typename Pre = PdNoPrefetch>
__device__ __forceinline__ void scan_solve(cpx<R> (&d)[MR], int len, int lt, int P,
                                           const cpx<R> *__restrict__ tb, cpx<R> *xw,
                                           Pre pre = Pre{}) {
  auto barrier = [] {
    if constexpr (LB)
      pd_lds_barrier();
    else
      __syncthreads();
  };
  auto fma = [](cpx<R> s, cpx<R> b, cpx<R> c) { return A::fma(s, b, c); };
  const cpx<R> zero = {R(0), R(0)};
  int lane = lt & 63;
  // lane passes through an empty asm: the shuffle indices derived from it
  // are formed here, not hoisted out of the caller's loop over work items
  // (where they would hold registers through the whole loop)
  asm volatile("" : "+v"(lane));
  const int wv = lt >> 6, NW = P >> 6;
  const cpx<R> r1 = tb[0], r2 = tb[1];
  // a wave with a ragged or empty chunk takes the masked loops
  const bool ragged = __any(len < MR);

  // forward recurrence inside the chunk, from zero: u_q
  cpx<R> acc = zero;
#pragma unroll
  for (int q = 0; q < MR; ++q) {
    acc = fma(d[q], r1, acc);
    d[q] = acc;
  }
  // scan of the chunk maps x -> R1 x + e_t across the wave (left to right):
  // lane l ends with R1^(l+1) and v at its chunk's last row from the wave's
  // start
  pre(0);   // the caller's next prefetch, a part at a time between the phases
  cpx<R> c = acc, m = tb[2];
  pd_scan_step<0x111, 0xF, A>(c, m);   // row_shr:1, 2, 4, 8
  pd_scan_step<0x112, 0xF, A>(c, m);
  pd_scan_step<0x114, 0xF, A>(c, m);
  pd_scan_step<0x118, 0xF, A>(c, m);
  pd_scan_step<0x142, 0xA, A>(c, m);   // row_bcast:15 into rows 1 and 3
  pd_scan_step<0x143, 0xC, A>(c, m);   // row_bcast:31 into rows 2 and 3
  cpx<R> ex = pd_dpp<0x138, 0xF>(c, zero);                // wave_shr:1
  const cpx<R> pl = pd_dpp<0x138, 0xF>(m, A::one());     // R1^lane
  const cpx<R> R64 = pd_readlane(m, 63);                  // R1^64
  if (lane == 63) xw[wv] = c;
  // sum_{q<len} r^q u_q by Horner, and sum_{q<len} r^(2q+1)
  cpx<R> h = zero, K = tb[6];
  if (!ragged) {
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) h = fma(d[q], r1, h);
  } else {
    // full chunks, the one ragged chunk (len = n mod MR), empty chunks
    K = pd_sel(len == MR, tb[6], pd_sel(len > 0, tb[8 + MR], zero));
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) h = pd_sel(q < len, fma(d[q], r1, h), h);
  }
  // R1^lt = r^s0: the power r^i at the chunk's start
  cpx<R> a0 = pl;
  if (wv & 1) a0 = A::mul(a0, R64);
  if (wv & 6) {
    const cpx<R> R128 = A::mul(R64, R64);
    if (wv & 2) a0 = A::mul(a0, R128);
    if (wv & 4) a0 = A::mul(a0, A::mul(R128, R128));
  }
  barrier();
  pre(1);
  // carry into this wave: the waves before it, in order
  {
    cpx<R> C = zero;
    for (int w = 0; w < wv; ++w) C = fma(xw[w], R64, C);
    ex = fma(ex, pl, C);   // v at the row before this chunk
  }
  // this chunk's share of z_0 = sum_i r^i v_i, summed over the group
  cpx<R> dot = A::mul(a0, fma(h, ex, K));
  // wave sum: row sums by row_shr, then the row totals into lane 63
  dot = cadd(dot, pd_dpp<0x111, 0xF>(dot, zero));
  dot = cadd(dot, pd_dpp<0x112, 0xF>(dot, zero));
  dot = cadd(dot, pd_dpp<0x114, 0xF>(dot, zero));
  dot = cadd(dot, pd_dpp<0x118, 0xF>(dot, zero));
  dot = cadd(dot, pd_dpp<0x142, 0xA>(dot, zero));
  dot = cadd(dot, pd_dpp<0x143, 0xC>(dot, zero));
  if (lane == 63) xw[NW + wv] = dot;
  barrier();
  pre(2);
  cpx<R> z0 = zero;
  for (int w = 0; w < NW; ++w) z0 = cadd(z0, xw[NW + w]);
  // rows of v - beta z_0 r^i = u_q + r^q (r ex - beta z_0 r^s0)
  {
    const cpx<R> E = csub(A::mul(r1, ex), A::mul(A::mul(tb[5], z0), a0));
    if (!ragged) {
#pragma unroll
      for (int q = 0; q < MR; ++q) d[q] = fma(d[q], tb[7 + q], E);
    } else {
#pragma unroll
      for (int q = 0; q < MR; ++q) d[q] = pd_sel(q < len, fma(d[q], tb[7 + q], E), zero);
    }
  }
  // backward recurrence inside the chunk, from zero
  acc = zero;
#pragma unroll
  for (int q = MR - 1; q >= 0; --q) {
    acc = fma(d[q], r2, acc);
    d[q] = acc;
  }
  // the same scan from the right: lane l ends with R2^(64-l) and the
  // value at its chunk's first row from the wave's end
  pre(3);
  cpx<R> cz = acc;
  m = tb[3];
  pd_scan_step<0x101, 0xF, A>(cz, m);   // row_shl:1, 2, 4, 8
  pd_scan_step<0x102, 0xF, A>(cz, m);
  pd_scan_step<0x104, 0xF, A>(cz, m);
  pd_scan_step<0x108, 0xF, A>(cz, m);
  // across rows (lane shuffles): rows 0 and 2 take the next row's first
  // lane, then rows 0 and 1 take lane 32
  {
    auto from = [](cpx<R> v, int l) { return cpx<R>{__shfl(v.re, l, 64), __shfl(v.im, l, 64)}; };
    const int srcA = (lane | 15) + 1;
    const cpx<R> oz = from(cz, srcA & 63), om = from(m, srcA & 63);
    const bool in = ((lane >> 4) & 1) == 0;
    cz = pd_sel(in, fma(cz, m, oz), cz);
    m = pd_sel(in, A::mul(m, om), m);
    const cpx<R> oz2 = from(cz, 32), om2 = from(m, 32);
    const bool in2 = lane < 32;
    cz = pd_sel(in2, fma(cz, m, oz2), cz);
    m = pd_sel(in2, A::mul(m, om2), m);
  }
  cpx<R> exz = pd_dpp<0x130, 0xF>(cz, zero);               // wave_shl:1
  const cpx<R> pr = pd_dpp<0x130, 0xF>(m, A::one());      // R2^(63-lane)
  const cpx<R> S64 = pd_readlane(m, 0);                    // R2^64
  if (lane == 0) xw[2 * NW + wv] = cz;
  barrier();
  {
    cpx<R> CZ = zero;
    for (int w = NW - 1; w > wv; --w) CZ = fma(xw[2 * NW + w], S64, CZ);
    exz = fma(exz, pr, CZ);   // the value at the row after this chunk
  }
  // rows: the local value plus r^(MR-q) times the value after the chunk
  if constexpr (SCALE) {
    const cpx<R> ik = tb[4];
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) d[q] = A::mul(ik, fma(d[q], tb[7 + MR - q], exz));
  } else {
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) d[q] = fma(d[q], tb[7 + MR - q], exz);
  }
}

// The same solve for groups of P <= 64 threads inside one wave (several
// systems per wave when P < 64): the scans and the sum for z_0 stay inside
// the group's lanes (shuffles of width P), so no LDS and no barrier.  tb may
// differ between groups (an LDS or global pointer per group).
template <typename R, int MR, typename A, bool SCALE>
__device__ __forceinline__ void scan_solve_group(cpx<R> (&d)[MR], int len, int lt, int P,
                                                 const cpx<R> *tb) {
  auto fma = [](cpx<R> s, cpx<R> b, cpx<R> c) { return A::fma(s, b, c); };
  auto shup = [P](cpx<R> v, int s) {
    return cpx<R>{__shfl_up(v.re, s, P), __shfl_up(v.im, s, P)};
  };
  auto shdn = [P](cpx<R> v, int s) {
    return cpx<R>{__shfl_down(v.re, s, P), __shfl_down(v.im, s, P)};
  };
  const cpx<R> zero = {R(0), R(0)};
  const cpx<R> r1 = tb[0], r2 = tb[1];
  const bool ragged = __any(len < MR);

  cpx<R> acc = zero;
#pragma unroll
  for (int q = 0; q < MR; ++q) {
    acc = fma(d[q], r1, acc);
    d[q] = acc;
  }
  cpx<R> c = acc, m = tb[2];
  for (int s = 1; s < P; s <<= 1) {
    const cpx<R> oc = shup(c, s), om = shup(m, s);
    const bool in = lt >= s;
    c = pd_sel(in, fma(c, m, oc), c);
    m = pd_sel(in, A::mul(m, om), m);
  }
  const cpx<R> ex = pd_sel(lt > 0, shup(c, 1), zero);       // v at the row before the chunk
  const cpx<R> a0 = pd_sel(lt > 0, shup(m, 1), A::one());   // R1^lt = r^s0
  cpx<R> h = zero, K = tb[6];
  if (!ragged) {
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) h = fma(d[q], r1, h);
  } else {
    // full chunks, the one ragged chunk (len = n mod MR), empty chunks
    K = pd_sel(len == MR, tb[6], pd_sel(len > 0, tb[8 + MR], zero));
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) h = pd_sel(q < len, fma(d[q], r1, h), h);
  }
  cpx<R> z0 = A::mul(a0, fma(h, ex, K));
  for (int s = P >> 1; s >= 1; s >>= 1)
    z0 = cadd(z0, cpx<R>{__shfl_xor(z0.re, s, P), __shfl_xor(z0.im, s, P)});
  {
    const cpx<R> E = csub(A::mul(r1, ex), A::mul(A::mul(tb[5], z0), a0));
    if (!ragged) {
#pragma unroll
      for (int q = 0; q < MR; ++q) d[q] = fma(d[q], tb[7 + q], E);
    } else {
#pragma unroll
      for (int q = 0; q < MR; ++q) d[q] = pd_sel(q < len, fma(d[q], tb[7 + q], E), zero);
    }
  }
  acc = zero;
#pragma unroll
  for (int q = MR - 1; q >= 0; --q) {
    acc = fma(d[q], r2, acc);
    d[q] = acc;
  }
  cpx<R> cz = acc;
  m = tb[3];
  for (int s = 1; s < P; s <<= 1) {
    const cpx<R> oz = shdn(cz, s), om = shdn(m, s);
    const bool in = lt + s < P;
    cz = pd_sel(in, fma(cz, m, oz), cz);
    m = pd_sel(in, A::mul(m, om), m);
  }
  const cpx<R> exz = pd_sel(lt + 1 < P, shdn(cz, 1), zero);   // the row after the chunk
  if constexpr (SCALE) {
    const cpx<R> ik = tb[4];
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) d[q] = A::mul(ik, fma(d[q], tb[7 + MR - q], exz));
  } else {
#pragma unroll
    for (int q = MR - 1; q >= 0; --q) d[q] = fma(d[q], tb[7 + MR - q], exz);
  }
}

// The table above for one frequency (host).  a, b, c: the constant sub-,
// main and super-diagonal; real: the system is real (lambda real), so the
// discriminant is clamped at zero and every entry is real.  Computed in long
// double and rounded once.
inline void pd_scan_table(std::complex<double> a, std::complex<double> b, std::complex<double> c,
                          bool real, int n, int MR, std::complex<double> *dst) {
  using C = std::complex<long double>;
  const C A(a.real(), a.imag()), B(b.real(), b.imag()), Cc(c.real(), c.imag());
  C kap;
  if (real) {
    long double disc = B.real() * B.real() - 4.0L * A.real() * Cc.real();
    if (disc < 0.0L) disc = 0.0L;
    const long double s = std::sqrt(disc);
    kap = C(B.real() >= 0.0L ? (B.real() + s) / 2.0L : (B.real() - s) / 2.0L, 0.0L);
  } else {
    const C s = std::sqrt(B * B - 4.0L * A * Cc);
    const C k1 = (B + s) / 2.0L, k2 = (B - s) / 2.0L;
    kap = std::abs(k1) >= std::abs(k2) ? k1 : k2;
  }
  const C r1 = -A / kap, r2 = -Cc / kap, rho = r1 * r2;
  auto put = [&](int i, C v) { dst[i] = std::complex<double>((double)v.real(), (double)v.imag()); };
  C R1 = 1.0L, R2 = 1.0L;
  for (int q = 0; q < MR; ++q) {
    R1 *= r1;
    R2 *= r2;
  }
  put(0, r1);
  put(1, r2);
  put(2, R1);
  put(3, R2);
  // w_0 = sum_{m < n} rho^m by doubling: (S, rho^m) for the bits of n
  C S = 0.0L, pm = 1.0L, Sb = 1.0L, pb = rho;
  for (int m = n; m; m >>= 1) {
    if (m & 1) {
      S += pm * Sb;
      pm *= pb;
    }
    Sb += pb * Sb;
    pb *= pb;
  }
  const C ik = 1.0L / kap, beta = rho / (1.0L + rho * S);
  put(4, ik);
  put(5, beta);
  C K = 0.0L, p = r1;
  for (int q = 0; q < MR; ++q) {
    K += p;
    p *= rho;
  }
  put(6, K);
  C pq = 1.0L;
  for (int q = 0; q <= MR; ++q) {
    put(7 + q, pq);
    pq *= r1;
  }
  C Kr = 0.0L, pr = r1;
  for (int q = 0; q < n % MR; ++q) {
    Kr += pr;
    pr *= rho;
  }
  put(8 + MR, Kr);
}
