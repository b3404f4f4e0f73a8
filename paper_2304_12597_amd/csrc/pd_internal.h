// Internal declarations shared by the HIP sources of libparadiag.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/paradiag.h"
#include <rocprofiler-sdk-roctx/roctx.h>

// ---------------------------------------------------------------------------
// complex helpers (interleaved re/im, real type R = double or float)
// ---------------------------------------------------------------------------
template <typename R> struct cpx { R re, im; };

template <typename R> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };

template <typename R>
__device__ __forceinline__ cpx<R> cmk(R re, R im) { return cpx<R>{re, im}; }
template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.re, -a.im}; }
// a - b*c
template <typename R>
__device__ __forceinline__ cpx<R> cfms(cpx<R> a, cpx<R> b, cpx<R> c) {
  return {a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re};
}
template <typename R>
__device__ __forceinline__ cpx<R> crecip(cpx<R> a) {
  R d = R(1) / (a.re * a.re + a.im * a.im);
  return {a.re * d, -a.im * d};
}
template <typename R>
__device__ __forceinline__ cpx<R> cneg(cpx<R> a) { return {-a.re, -a.im}; }
// c ? a : b, one component at a time (a select of whole structs can end up as
// a select of stack addresses)
__device__ __forceinline__ double pd_sel(bool c, double a, double b) { return c ? a : b; }
template <typename R>
__device__ __forceinline__ cpx<R> pd_sel(bool c, cpx<R> a, cpx<R> b) {
  return cpx<R>{c ? a.re : b.re, c ? a.im : b.im};
}
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV>
__device__ __forceinline__ cpx<R> cmul_mi(cpx<R> a) {
  return INV ? cpx<R>{-a.im, a.re} : cpx<R>{a.im, -a.re};
}

// The capacitance GMRES stops at residual <= PD_GMRES_TOL_FACTOR * tol * ||b||:
// the error in x reaches U through the shifted solves of the last pass, which
// amplify it on ill-conditioned problems (small diffusion, long horizons).
constexpr double PD_GMRES_TOL_FACTOR = 1e-2;

// GMRES target for a solve to tol in precision prec.  With float32 shifted
// solves the capacitance products carry float32 rounding, so a GMRES residual
// below about 1e-7 of ||b|| is not resolved by them: iterations past it only
// refine the Krylov estimate (the mixed form's float64 refinement corrects
// what remains), so the target is floored there.
inline double pd_gmres_tol(int prec, double tol) {
  const double t = tol * PD_GMRES_TOL_FACTOR;
  return (prec != PD_FP64 && t < 1e-7) ? 1e-7 : t;
}

// LDS column layout of the time and DST transforms: entry i of a column sits
// at pd_fpad(i) = i + i/8, which spreads the power-of-two strides of the
// Stockham stages over all LDS banks; columns are pd_fft_col_stride(N)
// entries apart (odd, so that columns start on different banks).
__host__ __device__ __forceinline__ int pd_fpad(int i) { return i + (i >> 3); }
__host__ __device__ __forceinline__ int pd_fft_col_stride(int N) {
  const int s = pd_fpad(N - 1) + 1;
  return s | 1;
}
// Twiddles of a length-N transform in LDS: lo[m] = w^m for m < min(N, 64) and
// hi[h] = w^(64 h) for h < max(N / 64, 1); w^m = hi[m / 64] lo[m % 64].
__host__ __device__ __forceinline__ int pd_tw_lo(int N) { return N < 64 ? N : 64; }
__host__ __device__ __forceinline__ int pd_tw_entries(int N) {
  return pd_tw_lo(N) + (N < 64 ? 1 : N / 64);
}

// ---------------------------------------------------------------------------
// batched launches: one entry per problem, a block map (problem, local block)
// ---------------------------------------------------------------------------
struct FftJob {
  int N, n, nbar, dims, C, stride;
  double tau;
  const double *u0, *F, *U, *coef, *dal;
  const void *tw;
  void *spec;
  double *out;
  double *red;
};

struct TriJob {
  int n, F2, P, spb, nitems, nblk, has_mass;
  double ml, md, mu, kl, kd, ku;   // constant diagonals of M and tau K
  const double *coef64;
  const void *lam, *fac;
  const double *gw;
  const void *in;
  const double *vin, *xv;
  double wscale;
  void *out;
  double *partials;
  const double *skip;   // nonzero: the problem's GMRES has converged (J jobs)
  int scan;             // the recurrence-form solve (pd_scan.h), P >= 64 float64 only
};

struct VecJob {     // one problem's vectors for the batched GMRES kernels
  int n, B;         // vector length, vector-kernel blocks
  int G;            // partial rows of the shifted-solve reductions
  double *V, *w, *x, *red1, *red2, *gm, *partials, *bout;
  const double *b;
  const double *done;   // the problem's GMRES converged flag
};

// Direct global -> LDS load of 16 bytes per lane (gfx950 global_load_lds):
// lane j of the wave writes lds_base + 16 j; lds_base must be wave-uniform.
// Completion is tracked by the vector-memory counter (wait with
// __builtin_amdgcn_s_waitcnt before a barrier).
__device__ __forceinline__ void pd_lds_dma16(const void *gptr, void *lds_base) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(gptr, lds_base, 16, 0, 0);
#endif
}
__device__ __forceinline__ void pd_lds_dma4(const void *gptr, void *lds_base) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(gptr, lds_base, 4, 0, 0);
#endif
}
__device__ __forceinline__ void pd_wait_all() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_s_waitcnt(0);
#endif
}
// Block barrier for data exchanged through LDS by ds_read / ds_write only.
// __syncthreads() is a release/acquire fence as well, so it waits for every
// outstanding vector-memory operation of the wave -- including a
// global_load_lds prefetch into a different LDS area, which then no longer
// overlaps anything.  This barrier waits only for the wave's LDS accesses
// (lgkmcnt(0); vmcnt and expcnt left at their maxima in the gfx9 encoding)
// and keeps the compiler from moving memory accesses across it.  LDS that a
// prefetch writes must still be read only after pd_wait_all() and a full
// barrier.
__device__ __forceinline__ void pd_lds_barrier() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
#endif
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct TriConfig {
  int P;        // threads per system (power of two)
  int MR;       // rows per thread
  int spb;      // systems per block
  int block;    // threads per block = P * spb
  size_t lds;   // dynamic LDS bytes
  int pipe;     // complex128, P >= 64: the pipelined uniform body
};

struct Line2DConfig {
  int MR = 8, P = 1, S = 1, block = 1, mgroups = 1, nkc = 1, kchunk = 1;
  size_t lds = 0;
};

// The chunked capacitance product (capprod.hip): chunking and the offsets
// (doubles) of its tables and workspace in one device buffer.
struct CpLayout {
  int m = 0, nc = 0, L = 0, N0 = 0, NL = 0;
  int Q = 0;        // matrix-core steps over a chunk window (4 Q >= N0 + 2)
  int NT = 0, NTc = 0, NH = 0;   // column tiles of 16 chunks, their chunks, blocks over them
  int VL = 0;       // doubles of v staged in LDS
  int G1 = 0;       // frequency groups of 4 (tables)
  int G1run = 0;    // blocks of the first launch (G1, or G1 - 1 with the real pair)
  int pair = 0;     // frequencies 0 and F2 - 1 share slot 0 of the first block
  int k0sep = 0;    // frequency 0 goes through the shifted-solve kernel (see pd_cp_tables)
  int MT = 0;       // row tiles of 16
  int Sk = 0, KPS = 0, KPT = 0;  // frequency splits, frequencies per split, rows
  int HLS = 0, NV = 0;   // last-chunk window; vector rows (last chunk's rows, chunks' last rows)
  int local = 0;    // the chunk-local term is nonzero (some rho_i != 0)
  size_t T1 = 0, hL = 0, red = 0, gk = 0, T3 = 0, c1 = 0, T4 = 0, L1h = 0, gJ0 = 0;
  size_t tables = 0, U = 0, tiles = 0, vrow = 0, total = 0;
};

// One problem's capacitance-product launches (device-readable; the batched
// launches read an array of them).
struct CpJob {
  int n = 0, F2 = 0, pair = 0, m = 0, nc = 0, L = 0, Q = 0, NTc = 0, VL = 0, MT = 0;
  int Sk = 0, KPS = 0, KPT = 0, NH = 0, HLS = 0, S = 0;
  double md = 0, ml = 0;
  const double *v = nullptr;    // input (batched: the GMRES basis, v = V + jv n)
  double *out = nullptr;        // J v
  const double *T1 = nullptr, *T3 = nullptr, *T4 = nullptr, *L1h = nullptr;
  const cpx<double> *hL = nullptr, *red = nullptr, *c1 = nullptr, *gk = nullptr;
  cpx<double> *U = nullptr;
  double *tiles = nullptr, *vrow = nullptr;
  const double *skip = nullptr; // stop flag (nonzero: no product)
  const double *extra = nullptr; // the k = 0 term added by the last launch, or null
};

struct pd_plan_s {
  int n = 0, ell = 0, dims = 1, nbar = 0, F2 = 0;
  double tau = 0, alpha = 1, w = 1;   // w = alpha^(1/ell)
  int prec = PD_FP64;
  int maxit = 64, max_sweeps = 16, check_residual = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  bool mass_identity = true;
  // sqrt(ell (ell + 1) / 2) sqrt(lmax(M) / lmin(M)) when M is SPD and K SPSD
  // (Gershgorin), else -1: turns ||R||_F / ||M U||_F into an error bound
  double err_factor = -1.0;
  bool uniform = false;        // M and tau K have constant diagonals
  double uni[6] = {0, 0, 0, 0, 0, 0};  // ml md mu tkl tkd tku when uniform

  // host constants (float64)
  std::vector<double> lam;     // 2*F2: lambda_k = 1 - pi_k
  std::vector<double> gB;      // 2*F2: weight_k * gamma_k (b reduction)
  std::vector<double> gJ;      // 2*F2: w * weight_k * gamma_k (J product)

  // device constants
  double *coef64 = nullptr;    // 6*n: ML MD MU tKL tKD tKU (1D) ; 2D: T row
  float *coef32 = nullptr;     // same, float
  double *lam64 = nullptr;     // 2*F2
  float *lam32 = nullptr;
  double *gB64 = nullptr, *gJ64 = nullptr;  // 2*F2 each
  double *tw64 = nullptr;      // 2*ell: exp(-2 pi i m / ell)
  float *tw32 = nullptr;
  double *dal = nullptr;       // 2*ell: alpha^(t/ell), alpha^(-t/ell)
  double *fac64 = nullptr;     // uniform-path elimination factors (float64)
  float *fac32 = nullptr;      // the same rounded to float

  // workspace
  void *spec = nullptr;        // [F2][nbar] complex (c128 or c64)
  void *spec2 = nullptr;       // PD_MIXED: a second spectrum, so that the last
                               // correction's stays while the next residual is
                               // transformed (rollback on a stalled sweep)
  size_t spec_bytes = 0;
  size_t bytes = 0;            // device bytes this plan allocated
  double *partials = nullptr;  // [tri_G][nbar]
  double *rstage = nullptr;    // [ceil(G/16)][nbar] reduction slices
  double *host_dev = nullptr;  // device view of host_pin (kernel-written status)
  const double *gm_skip = nullptr;   // set during GMRES: converged flag for the J kernels
  int gm_pred = 2;             // GMRES iterations enqueued ahead (the last solve's count)
  int gm_seen = 0;             // a solve has run (gm_pred is learned)
  int autotune = 0;            // buffers sized for every tuning candidate
  int early_exit = 0;          // Algorithm 3's test on U_1 before the correction
  int krylov = 0;              // capacitance solver: 0 GMRES, 1 Algorithm 2
  int fom_q = 1;               // Algorithm 2: residual check every fom_q steps
  double *fom = nullptr;       // Algorithm 2 device state (pd_fom_doubles)
  void *fom_h = nullptr;       // Algorithm 2: -w h_i for all i (spectrum sized)
  // sine-basis shifted solves (symmetric Toeplitz M, K; n + 1 a power of two)
  int sine = 0;
  int sine_C = 1;              // rows per block of the DST-I kernel
  double *sine_q = nullptr;    // [n+1] sin(pi j / (n+1))
  double *sine_wN = nullptr;   // [(n+1)/2 + 1] exp(-2 pi i m / (n+1))
  double *sine_twH = nullptr;  // [(n+1)/2] exp(-2 pi i m / ((n+1)/2))
  double *sine_m = nullptr;    // [n] eigenvalues of M on the sine modes
  double *sine_k = nullptr;    // [n] eigenvalues of tau K on the sine modes
  int tri_G = 0;
  double *bvec = nullptr, *xvec = nullptr, *wvec = nullptr;
  double *V = nullptr;         // [(maxit+1)][ncap] Krylov basis
  double *gm = nullptr;        // GMRES small state (device)
  double *red = nullptr;       // reduction scratch
  int red_blocks = 0;
  double *host_pin = nullptr;  // pinned host scalars

  TriConfig tri;
  Line2DConfig l2d;
  int fft_C = 1;               // complex columns (point pairs) per FFT block
  int fft_stride = 0;          // LDS column stride (complex elements)
  int dst_C = 1;               // 2D: row pairs per DST-I block
  double *twd = nullptr;       // 2D: exp(-2 pi i m / (2(n+1))) twiddles
  int dst_L = 0;               // 2D: 0 if n + 1 is a power of two, else the
                               // chirp-z DST's FFT length L >= 2n - 1
  size_t twd_chirp = 0, twd_bhat = 0, twd_cos = 0;   // offsets (doubles) in twd
  double *wreal = nullptr;     // 2D: [ell][nbar] float64 work array (DST-x domain);
                               // BDF: the time-domain input of the transforms
  // BDF of order s (Section 5); s = 1 is backward Euler and uses none of these
  int bdf_s = 1;
  double bdf_beta = 1.0;
  double bdf_alpha[6] = {1, 0, 0, 0, 0, 0};   // alpha_1..alpha_s
  int ncap = 0;                // capacitance vector length: s * nbar
  double *wz = nullptr;        // BDF: capacitance-product partial sums
  double *bdf_g = nullptr;     // BDF: [s][F2] complex weight_f gamma_f^(k)
  double *bdf_h = nullptr;     // BDF 2D: [ell][nbar] h before the DST along x
  double *bdf_t = nullptr;     // BDF 2D: [s][nbar] rows in the DST-x domain
  // chunked capacitance product (1D, symmetric Toeplitz M and tau K): tables
  // and workspace in one buffer laid out by cpl
  int cp_on = 0;
  CpLayout cpl;
  double *cp_tab = nullptr;
};
constexpr int PD_BDF_GCH = 16;   // frequency chunks of the BDF capacitance product

// A named host range for profilers (roctx; shown by rocprofv3 --marker-trace):
// the stages of a solve as the host enqueues them.  A push and a pop per
// range, nothing else, when no profiler is attached.
struct PdRange {
  explicit PdRange(const char *name) { roctxRangePushA(name); }
  ~PdRange() { roctxRangePop(); }
  PdRange(const PdRange &) = delete;
  PdRange &operator=(const PdRange &) = delete;
};

// error reporting
void pd_set_error(const std::string &msg);
#define PD_HIP_CHECK(call)                                                   \
  do {                                                                       \
    hipError_t _e = (call);                                                  \
    if (_e != hipSuccess) {                                                  \
      pd_set_error(std::string(#call) + ": " + hipGetErrorString(_e));       \
      return PD_EHIP;                                                        \
    }                                                                        \
  } while (0)

// ---------------------------------------------------------------------------
// stage launchers (return PD_OK or an error code)
// ---------------------------------------------------------------------------
// forward time transform: mode 0 = h input, 1 = residual input (R = G - A(U),
// norms accumulated into red)
pd_status pd_launch_fft_forward(pd_plan p, const double *u0, const double *F,
                                const double *U, void *out, int mode);
// inverse: accumulate = 0 store, 1 add into U
pd_status pd_launch_fft_inverse(pd_plan p, const void *in, double *U,
                                int accumulate);
// shifted solves. mode 0: b-reduction of P^{-1} M Hhat (partials), 1: write
// Y = P^{-1} M (Hhat - w x), 2: J-product partials of P^{-1} M v.
pd_status pd_launch_tridiag(pd_plan p, int mode, const void *in,
                            const double *xv, void *out);
// 2D: orthonormal DST-I along x of every row. mode 0: h from (u0, F);
// 1: float64 residual of (u0, F, U) with norms in red; 2: in.
pd_status pd_launch_dst_x(pd_plan p, int mode, const double *u0, const double *F,
                          const double *U, const double *in, double *out, int accumulate);
int pd_choose_dst_C(int n);
int pd_dst_chirp_length(int n);
pd_status pd_launch_dst_rows1d(pd_plan p, int mode, const double *u0, const double *F,
                               const double *in, double *out);
Line2DConfig pd_choose_line2d(int n, int F2, int prec, int cus);
void pd_line2d_factors(const pd_plan p, std::vector<double> &fac);
pd_status pd_launch_line2d(pd_plan p, int mode, const void *in, const double *xv, void *out);
void pd_line2d_set_attributes(size_t max_lds);
// whole-pipeline helpers (1D or 2D)
pd_status pd_forward(pd_plan p, const double *u0, const double *F, const double *U, void *spec,
                     int residual);
pd_status pd_inverse(pd_plan p, const void *spec, double *U, int accumulate);
// 2D: orthonormal DST-I along x of trows time rows (in -> out, or added)
pd_status pd_launch_dst_x_rows(pd_plan p, const double *in, double *out, int trows,
                               int accumulate);
int pd_forward_norm_blocks(pd_plan p);
int pd_dst_blocks(pd_plan p);
// sum partials: out = base + sum_g partials[g]   (base may be NULL)
pd_status pd_launch_reduce_partials(pd_plan p, const double *base,
                                    double *out);
pd_status pd_capacitance_apply_impl(pd_plan p, const double *v, double *Jv);
// the chunked capacitance product (capprod.hip)
void pd_cp_chunking(int n, int *m, int *nc, int *L);
bool pd_cp_eligible(int n, int dims, int bdf_s, bool uniform, const double *uni);
CpLayout pd_cp_layout(int n, int F2);
void pd_cp_tables(pd_plan p, std::vector<double> &tab);
bool pd_cp_fits(int n, int F2, size_t max_lds);
void pd_cp_set_attributes(size_t max_lds);
pd_status pd_cp_apply(pd_plan p, const double *v, double *Jv);
// The job of plan p (input v, output Jv, stop flag skip) and, for batches,
// its launches' block counts (launch 1, 2, 3), block size of launch 2 and
// dynamic LDS bytes of launches 1 and 2.
CpJob pd_cp_job(pd_plan p, const double *v, double *Jv, const double *skip);
// k = 0 J-product term by one block of the shifted-solve kernel (partials row 0)
pd_status pd_launch_j_first_item(pd_plan p, const double *v, const double *gw);
int pd_cp_blocks(const CpJob &J, int launch);
int pd_cp_threads2(const CpJob &J);
size_t pd_cp_lds(const CpJob &J, int launch);
pd_status pd_cp_launch_batch(const CpJob *jobs, const int2 *map1, int nb1, const int2 *map2,
                             int nb2, int threads2, const int2 *map3, int nb3, size_t lds1,
                             size_t lds2, const int *active, int jv, hipStream_t s);
pd_status pd_gmres(pd_plan p, const double *b, double *x, double rtol,
                   int *iters, double *relres);
// rel = ||G - A(U)||_F / ||G||_F; est (if non-null): the plan's error bound
// from the same residual (pd_info.est_rel_error), or -1
pd_status pd_residual_impl(pd_plan p, const double *u0, const double *F,
                           const double *U, double *rel, double *est = nullptr);
pd_status pd_sum_norms(pd_plan p, int nblk, double *rn2, double *gn2);
// Algorithm 2 (fom.hip)
constexpr int PD_FOM_MAXM = 32;   // largest Krylov dimension of Algorithm 2
size_t pd_fom_doubles(int n, int F2);
size_t pd_fom_mfac_offset(int F2);
bool pd_fom_supported(pd_plan p);
pd_status pd_fom(pd_plan p, const double *b, double *x, double rtol, int *iters,
                 double *relres, int *checks);
void pd_fom_mass_factors(pd_plan p, std::vector<double> &out);
// BDF of order s > 1 (bdf.hip): h of eq. discrete_probBDF into out [ell][nbar];
// the block capacitance product J^(s) v; the whole solve; the float64
// residual norms ||G - A(U)||^2 and ||G||^2.
pd_status pd_bdf_rhs(pd_plan p, const double *u0s, const double *F, double *out);
pd_status pd_bdf_apply(pd_plan p, const double *v, double *Jv);
pd_status pd_bdf_solve(pd_plan p, const double *u0s, const double *F, double *U, double tol,
                       pd_info *info);
pd_status pd_bdf_residual_norms(pd_plan p, const double *u0s, const double *F,
                                const double *U, double *rn2, double *gn2);
int pd_bdf_residual_blocks(pd_plan p);
// Block Galerkin method for J^(s) (bgal.hip): basis dimension s m <= BG_SMAX;
// T is BG_TROWS x BG_LDT row-major.  Offsets (doubles) into p->fom.
constexpr int BG_SMAX = 32;
constexpr int BG_TROWS = BG_SMAX + 6;
constexpr int BG_LDT = BG_SMAX;
struct BgLayout {
  size_t T, beta, proj, E, L, part, G, y, cw, z, zpart, state, mpart, mfac, ctab, gtab, thtab,
      total;
};
BgLayout pd_bgal_layout(int n, int F2);
pd_status pd_bgal(pd_plan p, const double *b, double *x, double rtol, int *iters,
                  double *relres, int *checks);
// w = tau M^{-1} K v with the uniform mass factors mfac (Algorithm 2's operator;
// BDF plans: tau beta M^{-1} K)
pd_status pd_fom_apply(pd_plan p, const cpx<double> *mfac, const double *v, double *w);
// multi-block vector helpers (fom.hip): Gram-Schmidt against up to 39 basis
// vectors, normalisation, squared norms; the 2D operator in the DST-x domain
int pd_mvec_blocks(int n);
pd_status pd_mvec_orth(pd_plan p, int n, const double *V, double *w, int cnt, double *T, int ldT,
                       int col, double *part);
pd_status pd_mvec_normalize(pd_plan p, int n, double *V, const double *w, int cnt, double *T,
                            int ldT, int col, double *tout, double *part);
pd_status pd_mvec_norm2(pd_plan p, int n, const double *w, double *out, int acc, double *part);
pd_status pd_apply2d(pd_plan p, const double *v, double *w);
// sine-basis path (sine.hip)
int pd_sine_dst_C(int n, int ell);
size_t pd_sine_dst_lds(int n, int C);
size_t pd_sine_modal_lds(pd_plan p, int threads);
pd_status pd_launch_sine_dst(pd_plan p, int mode, const double *u0, const double *F,
                             const double *in, double *out);
pd_status pd_launch_sine_modal(pd_plan p, const double *A, double *B);
void pd_sine_set_attributes(size_t max_lds);
int pd_residual_blocks(pd_plan p);
// ||G - A(U)||_F^2, ||G||_F^2 and ||M U||_F^2 in float64 (synchronises)
pd_status pd_residual_norms(pd_plan p, const double *u0, const double *F, const double *U,
                            double *rn2, double *gn2, double *un2);
int pd_fft_blocks(pd_plan p);
int pd_vec_blocks(int n);
size_t pd_gmres_state_doubles(int maxit);
int pd_choose_fft_C(int ell, int nbar, int prec, size_t max_lds);
// Work items of a shifted-solve launch: the pipelined body pairs the two real
// shifts k = 0 and k = ell/2 into one item (slot 0), so F2 - 1 slots.
inline int pd_tri_nitems(const TriConfig &T, int F2) {
  const int slots = T.pipe ? F2 - 1 : F2;
  return (slots + T.spb - 1) / T.spb;
}

// The pipelined body solves symmetric Toeplitz systems (uniform 1D grids,
// M and tau K symmetric) by the recurrence form of pd_scan.h instead of the
// partition method; the plan's factor table then holds its constants.
inline bool pd_use_scan(const pd_plan p) {
  const double *u = p->uni;
  return p->dims == 1 && p->uniform && p->tri.pipe && p->tri.MR >= 8 && p->tri.P <= 512 &&
         p->tri.P % 64 == 0 && u[0] == u[2] && u[3] == u[5];
}

// The 2D line solves of float64 plans with groups of at most one wave use
// the recurrence form as well (symmetric Toeplitz lines, pd_scan.h).
inline bool pd_line2d_scan(const pd_plan p) {
  return p->dims == 2 && p->prec == PD_FP64 && p->l2d.P <= 64 && p->l2d.MR >= 4;
}

// Threads per shifted-solve block: 512 for complex128 (a 256-register budget
// per thread keeps the partition solve out of scratch), 1024 otherwise.
inline int pd_tri_block_threads(int prec) { return prec == PD_FP64 ? 512 : 1024; }
TriConfig pd_choose_tri(int n, int F2, int prec, size_t max_lds);
TriConfig pd_choose_tri_mr(int n, int F2, int prec, size_t max_lds, int MR);
void pd_uniform_factors(const pd_plan p, int MR, std::vector<double> &fac);
void pd_fft_set_attributes(size_t max_lds);
void pd_tri_set_attributes(size_t max_lds);


// batched stage launchers (all problems of one precision; blocks map to
// (problem, local block) pairs in `map`, int2 per block)
pd_status pd_launch_fft_forward_batch(int prec, const FftJob *jobs, const int2 *map, int nblocks,
                                      int threads, size_t lds, hipStream_t s);
pd_status pd_launch_fft_inverse_batch(int prec, const FftJob *jobs, const int2 *map, int nblocks,
                                      int threads, size_t lds, hipStream_t s);
pd_status pd_launch_tridiag_batch(int prec, int MR, int mode, const TriJob *jobs, const int2 *map,
                                  int nblocks, size_t lds, const int *active, int jv,
                                  hipStream_t s);
pd_status pd_launch_reduce_batch(const VecJob *jobs, const int2 *map, int nblocks, int base_j,
                                 const int *active, hipStream_t s);
void pd_fft_batch_set_attributes(size_t max_lds);
void pd_tri_batch_set_attributes(size_t max_lds);
// batched GMRES vector kernels (gmres.hip); vmap: blocks of every problem's
// vectors, one int2 (problem, block) each; pmap: one block per problem
pd_status pd_gmres_batch_dots(const VecJob *jobs, const int2 *vmap, int nvb, int nv, int which,
                              const int *active, hipStream_t s);
pd_status pd_gmres_batch_update(const VecJob *jobs, const int2 *vmap, int nvb, int nv, int j,
                                int MX, int pass, const int *active, hipStream_t s);
// one fused Arnoldi step per problem (vectors of at most pd_gmres_fused_max_n()
// entries): the single-problem path uses the same step
pd_status pd_gmres_batch_arnoldi(const VecJob *jobs, int count, int j, int MX, double rtol,
                                 double *status, const int *active, hipStream_t s);
int pd_gmres_fused_max_n();
// the fused start of GMRES per problem (beta, state reset, V_0), as alone
pd_status pd_gmres_batch_start(const VecJob *jobs, int count, int MX, double *status,
                               hipStream_t s);
// speculative capacitance GMRES of the single-problem 1D path
bool pd_gmres_fused_ok(pd_plan p);
size_t pd_gmres_done_index(int maxit);   // offset of the converged flag in the state
// drop cached batch runs (tables, captured graphs) that use this plan
void pd_batch_forget(pd_plan p);
pd_status pd_gmres_enqueue(pd_plan p, const double *b, double *x, double rtol, int count);
void pd_gmres_read(pd_plan p, int *m, double *res, double *beta, bool *done);
pd_status pd_gmres_continue(pd_plan p, double *x, double rtol, int *iters, double *relres);
pd_status pd_gmres_batch_givens(const VecJob *jobs, int count, int j, int MX, double *status,
                                const int *active, hipStream_t s);
pd_status pd_gmres_batch_init(const VecJob *jobs, int count, int MX, double *status,
                              hipStream_t s);
pd_status pd_gmres_batch_scale(const VecJob *jobs, const int2 *vmap, int nvb, int j, int MX,
                               int from_b, const int *active, hipStream_t s);
pd_status pd_gmres_batch_finish(const VecJob *jobs, const int2 *vmap, int nvb, int count, int MX,
                                const int *m_per_problem, hipStream_t s);
bool pd_batchable(const pd_plan *plans, int count);
pd_status pd_solve_batch_impl(const pd_plan *plans, int count, const double *const *u0,
                              const double *const *F, double *const *U, double tol,
                              pd_info *infos);

// Raise a kernel's dynamic-LDS limit to what the device allows beside its
// static LDS; failures are cleared so no stale error reaches the caller.
inline void pd_set_max_lds(const void *fn, int max_lds) {
  hipFuncAttributes a;
  int static_lds = 0;
  if (hipFuncGetAttributes(&a, fn) == hipSuccess) static_lds = (int)a.sharedSizeBytes;
  (void)hipGetLastError();
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds - static_lds);
  (void)hipGetLastError();
}
