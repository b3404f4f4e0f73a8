// Chunked tridiagonal solve shared by the shifted-solve kernels.
//
// A group of P threads solves one complex tridiagonal system whose rows have
// constant sub- and super-diagonals a, c and constant diagonal b (one
// frequency, one line).  Thread lt owns rows [lt*MR, lt*MR + len) held in
// d[] (len <= MR; rows past the end of the system are absent).  The
// elimination factors depend only on (a, b, c) and on the distance of a row
// from its chunk's ends, so they are precomputed (lfac, 6 complex values per
// distance 1..MR-1: upward pivot inverse rU, fill-ins ua and uc, downward
// pivot inverse rD, fill-in A and super-diagonal C) and each thread runs only
// the right-hand-side recurrences:
//
//   upward sweep    leaves row 0 as  x_0 + ua x_{prev last} + uc x_last = ud
//   downward sweep  leaves the last row as  x_last + A x_0 + C x_{next 0} = D
//
// Eliminating the first-row unknowns gives a P x P tridiagonal system in the
// chunks' last unknowns, solved by parallel cyclic reduction through LDS
// (xch, P Row3 entries per group).  A back substitution recovers the interior
// rows.  Unknowns before row 0 or after the last row are zero ghosts.
//
// Every thread of the block must call this together (it contains block
// barriers); on entry the block may still be reading its staging area, which
// xch is allowed to alias.  LB: the barriers only order LDS accesses
// (pd_lds_barrier), so that a global_load_lds prefetch issued before the call
// keeps streaming in; for callers whose xch does not alias LDS that such a
// prefetch writes.
#pragma once
#include "pd_internal.h"

template <typename R>
struct Row3 {
  cpx<R> a, c, d;   // normalised row:  a x_lo + x + c x_hi = d
};

// Arithmetic of one complex system ...
template <typename R>
struct CplxOps {
  static __device__ __forceinline__ cpx<R> mul(cpx<R> a, cpx<R> b) { return cmul(a, b); }
  static __device__ __forceinline__ cpx<R> fms(cpx<R> a, cpx<R> b, cpx<R> c) {
    return cfms(a, b, c);
  }
  static __device__ __forceinline__ cpx<R> recip(cpx<R> a) { return crecip(a); }
  static __device__ __forceinline__ cpx<R> one() { return cpx<R>{R(1), R(0)}; }
  // s + b*c, one expression per component (fused multiply-adds)
  static __device__ __forceinline__ cpx<R> fma(cpx<R> s, cpx<R> b, cpx<R> c) {
    return cpx<R>{s.re + b.re * c.re - b.im * c.im, s.im + b.re * c.im + b.im * c.re};
  }
};
// ... or of two independent real systems held in the real and imaginary
// parts (the real shifts k = 0 and k = ell/2 share one work item)
template <typename R>
struct DualOps {
  static __device__ __forceinline__ cpx<R> mul(cpx<R> a, cpx<R> b) {
    return cpx<R>{a.re * b.re, a.im * b.im};
  }
  static __device__ __forceinline__ cpx<R> fms(cpx<R> a, cpx<R> b, cpx<R> c) {
    return cpx<R>{a.re - b.re * c.re, a.im - b.im * c.im};
  }
  static __device__ __forceinline__ cpx<R> recip(cpx<R> a) {
    return cpx<R>{R(1) / a.re, R(1) / a.im};
  }
  static __device__ __forceinline__ cpx<R> one() { return cpx<R>{R(1), R(1)}; }
  static __device__ __forceinline__ cpx<R> fma(cpx<R> s, cpx<R> b, cpx<R> c) {
    return cpx<R>{s.re + b.re * c.re, s.im + b.im * c.im};
  }
};

template <typename R, int MR, typename A = CplxOps<R>, bool LB = false>
__device__ __forceinline__ void partition_solve(cpx<R> (&d)[MR], int len, int lt, int P,
                                                const cpx<R> *lfac, Row3<R> *xch,
                                                cpx<R> ca, cpx<R> cc) {
  auto barrier = [] {
    if constexpr (LB)
      pd_lds_barrier();
    else
      __syncthreads();
  };
  const cpx<R> zero = {R(0), R(0)};
  const int L2 = len < 2 ? 2 : len;   // a lone row gets a zero pad row
  cpx<R> ud = zero;
#pragma unroll
  for (int q = MR - 2; q >= 0; --q) {
    if (q <= L2 - 2) {
      const int dl = L2 - 1 - q;
      const cpx<R> r = lfac[(dl - 1) * 6 + 0];
      ud = (dl == 1) ? A::mul(d[q], r) : A::mul(A::fms(d[q], cc, ud), r);
    }
  }
  cpx<R> ua = lfac[(L2 - 2) * 6 + 1], uc = lfac[(L2 - 2) * 6 + 2];
  cpx<R> Ae = zero, Ce = zero, De = zero;
#pragma unroll
  for (int q = 1; q < MR; ++q) {
    if (q < len) {
      const cpx<R> r = lfac[(q - 1) * 6 + 3];
      d[q] = (q == 1) ? A::mul(d[q], r) : A::mul(A::fms(d[q], ca, d[q - 1]), r);
      if (q == len - 1) {
        Ae = lfac[(q - 1) * 6 + 4];
        Ce = lfac[(q - 1) * 6 + 5];
        De = d[q];
      }
    }
  }
  if (len == 0) { ua = zero; uc = zero; ud = zero; }

  barrier();   // staging area -> exchange area
  xch[lt] = Row3<R>{ua, uc, ud};
  barrier();
  Row3<R> nx = xch[lt + 1 < P ? lt + 1 : lt];
  const bool hasnx = lt + 1 < P;
  nx.a = pd_sel(hasnx, nx.a, zero);
  nx.c = pd_sel(hasnx, nx.c, zero);
  nx.d = pd_sel(hasnx, nx.d, zero);
  cpx<R> al = cneg(A::mul(Ae, ua));
  cpx<R> be = csub(csub(A::one(), A::mul(Ae, uc)), A::mul(Ce, nx.a));
  cpx<R> ga = cneg(A::mul(Ce, nx.c));
  cpx<R> de = csub(csub(De, A::mul(Ae, ud)), A::mul(Ce, nx.d));
  {
    const cpx<R> rb = A::recip(be);
    al = A::mul(al, rb);
    ga = A::mul(ga, rb);
    de = A::mul(de, rb);
  }
  for (int st = 1; st < P; st <<= 1) {
    barrier();
    xch[lt] = Row3<R>{al, ga, de};
    barrier();
    Row3<R> lo = xch[lt >= st ? lt - st : lt];
    Row3<R> hi = xch[lt + st < P ? lt + st : lt];
    const bool haslo = lt >= st, hashi = lt + st < P;
    lo.a = pd_sel(haslo, lo.a, zero); lo.c = pd_sel(haslo, lo.c, zero); lo.d = pd_sel(haslo, lo.d, zero);
    hi.a = pd_sel(hashi, hi.a, zero); hi.c = pd_sel(hashi, hi.c, zero); hi.d = pd_sel(hashi, hi.d, zero);
    const cpx<R> nb = csub(csub(A::one(), A::mul(al, lo.c)), A::mul(ga, hi.a));
    const cpx<R> nd = csub(csub(de, A::mul(al, lo.d)), A::mul(ga, hi.d));
    const cpx<R> na = cneg(A::mul(al, lo.a));
    const cpx<R> ng = cneg(A::mul(ga, hi.c));
    const cpx<R> rb = A::recip(nb);
    al = A::mul(na, rb);
    ga = A::mul(ng, rb);
    de = A::mul(nd, rb);
  }
  const cpx<R> xe = pd_sel(len >= 2, de, zero);
  barrier();
  xch[lt].d = xe;
  barrier();
  const cpx<R> xprev = pd_sel(lt > 0, xch[lt > 0 ? lt - 1 : 0].d, zero);
  const cpx<R> xs = csub(csub(ud, A::mul(ua, xprev)), A::mul(uc, xe));
  cpx<R> ynext = xe;
#pragma unroll
  for (int q = MR - 2; q >= 1; --q) {
    if (q <= len - 2) {
      d[q] = csub(csub(d[q], A::mul(lfac[(q - 1) * 6 + 4], xs)), A::mul(lfac[(q - 1) * 6 + 5], ynext));
      ynext = d[q];
    }
  }
  d[0] = xs;
#pragma unroll
  for (int q = 1; q < MR; ++q)
    if (q == len - 1) d[q] = xe;
}

// Elimination factors for constant (a, b, c), distances 1..MR-1, in the
// layout partition_solve expects (host, float64).
inline void pd_partition_factors(double ar, double ai, double br, double bi, double cr,
                                 double ci, int MR, double *dst /* 12*(MR-1) doubles */) {
  struct C { double re, im; };
  auto mul = [](C x, C y) { return C{x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re}; };
  auto sub = [](C x, C y) { return C{x.re - y.re, x.im - y.im}; };
  auto inv = [](C x) { double s = 1.0 / (x.re * x.re + x.im * x.im); return C{x.re * s, -x.im * s}; };
  const C a{ar, ai}, b{br, bi}, c{cr, ci};
  C rU = inv(b), ua = mul(a, rU), uc = mul(c, rU);
  C rD = rU, A = ua, Cc = uc;
  for (int dist = 1; dist < MR; ++dist) {
    if (dist > 1) {
      rU = inv(sub(b, mul(c, ua)));
      C nuc = mul(mul(c, uc), rU);
      uc = C{-nuc.re, -nuc.im};
      ua = mul(a, rU);
      rD = inv(sub(b, mul(a, Cc)));
      C nA = mul(mul(a, A), rD);
      A = C{-nA.re, -nA.im};
      Cc = mul(c, rD);
    }
    const C vals[6] = {rU, ua, uc, rD, A, Cc};
    double *o = dst + (size_t)(dist - 1) * 12;
    for (int j = 0; j < 6; ++j) {
      o[2 * j] = vals[j].re;
      o[2 * j + 1] = vals[j].im;
    }
  }
}
