// Plan creation: the constants of Algorithm 1 (Section 2) computed once in
// float64 on the host -- the circulant eigenvalues pi_k, the shifts
// lambda_k = 1 - pi_k, the weights gamma_k = F^{-T} e_ell (Appendix:
// gamma = conj(F) e_ell / ell, entries omega^(k)), the alpha-circulant
// scaling D_alpha (Section 4), DFT twiddles, the coefficients of M and tau K
// -- and the device workspace of every stage.
#include "pd_internal.h"
#include "pd_validate.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

namespace {
thread_local std::string g_last_error;

// exp(+2 pi i k / N) = (c, s), with exact values at multiples of pi/2 and
// octant reduction so that conjugate-symmetric tables are exactly symmetric.
void cis(long k, long N, double &c, double &s) {
  k %= N;
  if (k < 0) k += N;
  const long k4 = 4 * k;
  const long q = k4 / N;
  const long r = k4 - q * N;
  double cr, sr;
  if (2 * r <= N) {
    const double a = (M_PI / 2) * (double)r / (double)N;
    cr = std::cos(a);
    sr = std::sin(a);
  } else {
    const double a = (M_PI / 2) * (double)(N - r) / (double)N;
    cr = std::sin(a);
    sr = std::cos(a);
  }
  switch (q) {
    case 0: c = cr; s = sr; break;
    case 1: c = -sr; s = cr; break;
    case 2: c = -cr; s = -sr; break;
    default: c = sr; s = -cr; break;
  }
}

// Tables of the chirp-z DST-I of length n (N1 = n + 1), FFT length L:
// chirp[j] = exp(i pi j^2 / (2 N1)) for j = 0..n (j^2 reduced mod 4 N1), and
// bhat = (1/L) DFT_L of the wrapped conjugate chirp b[d mod L] = conj(c_|d|),
// |d| <= n - 1 (zero elsewhere), summed in long double.  Interleaved re, im.
void chirp_tables(int n, int L, double *chirp, double *bhat) {
  const long M = 4L * (n + 1);
  for (int j = 0; j <= n; ++j) {
    double c, s;
    cis(((long)j * j) % M, M, c, s);
    chirp[2 * j] = c;
    chirp[2 * j + 1] = s;
  }
  std::vector<double> wr(L), wi(L), br(L, 0.0), bi(L, 0.0);
  for (int m = 0; m < L; ++m) {
    double c, s;
    cis(m, L, c, s);
    wr[m] = c;    // exp(-2 pi i m / L)
    wi[m] = -s;
  }
  for (int d = -(n - 1); d <= n - 1; ++d) {
    const int q = d >= 0 ? d : d + L, a = d >= 0 ? d : -d;
    br[q] = chirp[2 * a];
    bi[q] = -chirp[2 * a + 1];
  }
  for (int k = 0; k < L; ++k) {
    long double sr = 0.0L, si = 0.0L;
    for (int d = -(n - 1); d <= n - 1; ++d) {
      const int q = d >= 0 ? d : d + L;
      const int m = (int)(((long)k * q) & (L - 1));
      sr += (long double)br[q] * wr[m] - (long double)bi[q] * wi[m];
      si += (long double)br[q] * wi[m] + (long double)bi[q] * wr[m];
    }
    bhat[2 * k] = (double)(sr / L);
    bhat[2 * k + 1] = (double)(si / L);
  }
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// BDF coefficients of order s <= 6 (Section 5, table of BDF coefficients):
// u_n - sum_j alpha_j u_{n-j} = tau beta f_n, as exact fractions.
void bdf_coefficients(int s, double *beta, double alpha[6]) {
  static const int num[6][7] = {{1, 1},
                                {2, 4, -1},
                                {6, 18, -9, 2},
                                {12, 48, -36, 16, -3},
                                {60, 300, -300, 200, -75, 12},
                                {60, 360, -450, 400, -225, 72, -10}};
  static const int den[6] = {1, 3, 11, 25, 137, 147};
  const int r = (s >= 1 && s <= 6) ? s - 1 : 0;
  *beta = (double)num[r][0] / den[r];
  for (int j = 0; j < 6; ++j) alpha[j] = (j <= r) ? (double)num[r][j + 1] / den[r] : 0.0;
}

template <typename T>
pd_status dev_alloc(T **ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return PD_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(ptr), count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    pd_set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    return PD_ENOMEM;
  }
  return PD_OK;
}

template <typename T>
pd_status upload(T *dst, const std::vector<T> &src, hipStream_t s) {
  if (src.empty()) return PD_OK;
  PD_HIP_CHECK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return PD_OK;
}

void free_plan(pd_plan p) {
  if (!p) return;
  void *ptrs[] = {p->coef64, p->coef32, p->lam64, p->lam32, p->gB64, p->gJ64, p->tw64,
                  p->tw32, p->dal, p->fac64, p->fac32, p->twd, p->wreal, p->spec, p->spec2, p->partials, p->rstage, p->bvec, p->xvec, p->wvec, p->V,
                  p->gm, p->red, p->sine_q, p->sine_wN, p->sine_twH, p->sine_m, p->sine_k,
                  p->fom, p->fom_h, p->wz, p->bdf_g, p->bdf_h, p->bdf_t, p->cp_tab};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  if (p->host_pin) (void)hipHostFree(p->host_pin);
  delete p;
}

size_t g_max_lds = 0;
int g_attr_device = -1;
std::mutex g_attr_mu;

// Launch configurations and device allocation sizes (in elements of their
// type) of a plan; shared by plan creation and paradiag_plan_bytes.
struct Layout {
  size_t coef = 0, lam = 0, tw = 0, dal = 0, fac = 0, twd = 0, wreal = 0, wz = 0, bdfg = 0,
         bdfh = 0, bdft = 0, sine = 0, fom = 0;
  size_t fom_h_bytes = 0;
  size_t cp = 0;   // chunked capacitance product: tables + workspace (doubles)
  size_t spec_bytes = 0, partials = 0, rstage = 0, vec = 0, V = 0, gm = 0, red = 0;
  size_t spec2_bytes = 0;   // PD_MIXED: the last correction's spectrum (stall rollback)
  size_t total_bytes() const {
    return coef * 12 + lam * 12 + 2 * lam * 8 + tw * 12 + dal * 8 + fac * 12 + twd * 8 +
           wreal * 8 + wz * 8 + bdfg * 8 + bdfh * 8 + bdft * 8 + spec_bytes + spec2_bytes + partials * 8 + rstage * 8 + 3 * vec * 8 + V * 8 + gm * 8 +
           red * 8 + sine * 8 + fom * 8 + fom_h_bytes + cp * 8;
  }
};

// Fills p->fft_C, fft_stride, tri, tri_G, l2d, dst_C; returns PD_OK or
// PD_ENOTSUP when a tile does not fit in LDS.
pd_status compute_layout(pd_plan p, int cus, size_t max_lds, Layout &L) {
  const int n = p->n, ell = p->ell, F2 = p->F2;
  const size_t cb = (p->prec == PD_FP64) ? 16 : 8;
  p->fft_C = pd_choose_fft_C(ell, p->nbar, p->prec, max_lds);
  p->fft_stride = pd_fft_col_stride(ell);
  if (((size_t)p->fft_C * p->fft_stride + pd_tw_entries(ell)) * cb > max_lds) {
    pd_set_error("time transform tile does not fit in LDS");
    return PD_ENOTSUP;
  }
  p->tri = pd_choose_tri(n, F2, p->prec, max_lds);
  if (p->dims == 1 && p->tri.lds > max_lds) {
    pd_set_error("shifted-solve tile does not fit in LDS");
    return PD_ENOTSUP;
  }
  if (!(p->dims == 1 && p->uniform)) p->tri.pipe = 0;
  const int nitems = pd_tri_nitems(p->tri, F2);
  p->tri_G = nitems < cus ? nitems : cus;
  L.partials = (size_t)p->tri_G * n;
  L.rstage = (size_t)(((p->autotune ? cus : p->tri_G) + 15) / 16) * n;
  if (p->dims == 2) {
    p->l2d = pd_choose_line2d(n, F2, p->prec, cus);
    if (p->l2d.lds > max_lds) {
      pd_set_error("2D line tile does not fit in LDS");
      return PD_ENOTSUP;
    }
    p->dst_L = pd_dst_chirp_length(n);   // 0: n + 1 a power of two
    const int ND = p->dst_L ? p->dst_L : 2 * (n + 1);
    p->dst_C = pd_choose_dst_C(n);
    if (((size_t)p->dst_C * pd_fft_col_stride(ND) + pd_tw_entries(ND)) * 16 > max_lds) {
      pd_set_error("DST tile does not fit in LDS");
      return PD_ENOTSUP;
    }
    L.fac = (size_t)F2 * n * 6 * (p->l2d.MR - 1) * 2;
    // twiddles of the DST's FFT length; for the chirp-z form the chirp c_j
    // (j = 0..n) and the transformed wrapped chirp; then cos(pi (j+1)/(n+1))
    p->twd_chirp = 2 * (size_t)ND;
    p->twd_bhat = p->twd_chirp + (p->dst_L ? 2 * (size_t)(n + 1) : 0);
    p->twd_cos = p->twd_bhat + (p->dst_L ? 2 * (size_t)p->dst_L : 0);
    L.twd = p->twd_cos + (size_t)n;
    L.wreal = (size_t)ell * p->nbar;
    if ((size_t)p->l2d.nkc * p->nbar > L.partials) L.partials = (size_t)p->l2d.nkc * p->nbar;
    L.rstage = std::max(L.rstage, (size_t)((p->l2d.nkc + 15) / 16) * p->nbar);
  } else if (p->uniform) {
    // + the paired real shifts; autotuning may pick up to 16 rows per thread
    L.fac = (size_t)(F2 + 1) * 6 * ((p->autotune ? 16 : p->tri.MR) - 1) * 2;
  }
  if (p->autotune) L.partials = std::max(L.partials, (size_t)cus * n);
  if (p->sine) {
    const int N = n + 1, H = N / 2;
    p->sine_C = pd_sine_dst_C(n, ell);
    if (pd_sine_dst_lds(n, p->sine_C) > max_lds) {
      pd_set_error("sine transform tile does not fit in LDS");
      return PD_ENOTSUP;
    }
    int need = p->fft_C * ell / 8;
    need = need < 64 ? 64 : need;
    if (pd_sine_modal_lds(p, ((need + 63) / 64) * 64) > max_lds) {
      pd_set_error("sine-basis time tile does not fit in LDS");
      return PD_ENOTSUP;
    }
    L.sine = (size_t)N + 2 * (size_t)(H + 1) + 2 * (size_t)H + 2 * (size_t)n;
    // n + 1 not a power of two: the DST of the time rows in chirp-z form, with
    // the 2D plans' table layout (twiddles of L, chirp, transformed chirp)
    p->dst_L = pd_dst_chirp_length(n);
    if (p->dst_L) {
      p->dst_C = pd_choose_dst_C(n);
      if (((size_t)p->dst_C * pd_fft_col_stride(p->dst_L) + pd_tw_entries(p->dst_L)) * 16 >
          max_lds) {
        pd_set_error("sine transform tile does not fit in LDS");
        return PD_ENOTSUP;
      }
      p->twd_chirp = 2 * (size_t)p->dst_L;
      p->twd_bhat = p->twd_chirp + 2 * (size_t)(n + 1);
      p->twd_cos = p->twd_bhat + 2 * (size_t)p->dst_L;
      L.twd = p->twd_cos;
    }
  }
  if (p->krylov == PD_KRYLOV_FOM) {
    L.fom = p->bdf_s > 1 ? pd_bgal_layout(p->nbar, F2).total : pd_fom_doubles(p->nbar, F2);
    L.fom_h_bytes = (size_t)p->bdf_s * F2 * p->nbar * cb;
  }
  if (p->bdf_s > 1) {
    L.wreal = (size_t)ell * p->nbar;
    L.wz = (size_t)PD_BDF_GCH * p->bdf_s * p->nbar;
    L.bdfg = 2 * (size_t)p->bdf_s * F2;
    if (p->dims == 2) {
      L.bdfh = (size_t)ell * p->nbar;
      L.bdft = (size_t)p->bdf_s * p->nbar;
    }
  }
  // float64 plans only: the reduced-precision forms keep their J-product in
  // the passes' own precision
  if (p->prec == PD_FP64 && pd_cp_eligible(n, p->dims, p->bdf_s, p->uniform, p->uni) &&
      pd_cp_fits(n, F2, max_lds)) {
    p->cp_on = 1;
    p->cpl = pd_cp_layout(n, F2);
    L.cp = p->cpl.total;
  }
  L.coef = 6 * (size_t)n;
  L.lam = 2 * (size_t)F2;
  L.tw = 2 * (size_t)ell;
  L.dal = 2 * (size_t)ell;
  L.spec_bytes = (size_t)F2 * p->nbar * cb;
  if (p->prec == PD_MIXED) L.spec2_bytes = L.spec_bytes;
  L.vec = p->ncap;
  L.V = (size_t)(p->maxit + 1) * p->ncap;
  L.gm = pd_gmres_state_doubles(p->maxit);
  const int B = pd_vec_blocks(p->ncap);
  size_t red_n = 2 * (size_t)B * (p->maxit + 2);
  size_t fb = 2 * (size_t)pd_fft_blocks(p);
  if (p->autotune) fb = 2 * (size_t)((p->nbar + 1) / 2);   // any tile width down to C = 1
  if (fb > red_n) red_n = fb;
  size_t rb = 3 * (size_t)pd_residual_blocks(p);
  if (rb > red_n) red_n = rb;
  if (p->bdf_s > 1) {
    size_t bb = 2 * (size_t)pd_bdf_residual_blocks(p);
    if (bb > red_n) red_n = bb;
  }
  if (p->dims == 2) {
    size_t db = 2 * (size_t)pd_dst_blocks(p);
    if (db > red_n) red_n = db;
  }
  L.red = red_n;
  return PD_OK;
}

}  // namespace

void pd_set_error(const std::string &msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// Autotuning (1D): the tile width C of the time transforms and the rows per
// thread MR of the shifted solves are timed on the plan's own buffers with
// zero inputs (run time does not depend on the values), the fastest kept,
// and the choice remembered per (n, ell, precision, constant diagonals or
// not) for later plans.  Buffers that depend on C or MR were sized for every candidate.
// ---------------------------------------------------------------------------
namespace {

struct TuneKey {
  int n, ell, prec, uniform;
  bool operator<(const TuneKey &o) const {
    if (n != o.n) return n < o.n;
    if (ell != o.ell) return ell < o.ell;
    if (prec != o.prec) return prec < o.prec;
    return uniform < o.uniform;
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tuned;   // -> (C, MR)

bool fft_C_ok(pd_plan p, int C, size_t max_lds) {
  const size_t cb = (p->prec == PD_FP64) ? 16 : 8;
  int maxC = 1;
  while (2 * maxC < p->nbar && maxC < 32) maxC *= 2;
  return C <= maxC && (size_t)C * p->ell / 8 <= 1024 &&
         ((size_t)C * p->fft_stride + pd_tw_entries(p->ell)) * cb <= max_lds;
}

// Shifted-solve configuration with MR rows per thread, factors uploaded;
// false if MR is not valid for this plan.
bool set_tri(pd_plan p, int MR, int cus, size_t max_lds) {
  TriConfig T = pd_choose_tri_mr(p->n, p->F2, p->prec, max_lds, MR);
  if (!(p->dims == 1 && p->uniform)) T.pipe = 0;
  if (T.lds > max_lds || T.block > (T.pipe ? 512 : 1024) || (T.pipe && MR == 16 && T.spb != 1))
    return false;
  p->tri = T;
  const int nitems = pd_tri_nitems(T, p->F2);
  p->tri_G = nitems < cus ? nitems : cus;
  if (p->uniform) {
    std::vector<double> fac;
    pd_uniform_factors(p, MR, fac);
    std::vector<float> fac32(fac.begin(), fac.end());
    if (hipMemcpy(p->fac64, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->fac32, fac32.data(), fac32.size() * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess)
      return false;
  }
  return true;
}

template <typename Fn>
float time_launches(pd_plan p, Fn fn) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.f;
  }
  fn();   // warm-up
  (void)hipEventRecord(e0, p->stream);
  for (int r = 0; r < 3; ++r) fn();
  (void)hipEventRecord(e1, p->stream);
  float ms = -1.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    ms = -1.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

pd_status autotune(pd_plan p, int cus, size_t max_lds) {
  const TuneKey key{p->n, p->ell, p->prec, p->uniform ? 1 : 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      p->fft_C = it->second.first;
      if (!set_tri(p, it->second.second, cus, max_lds)) {
        pd_set_error("autotune: cached shifted-solve configuration not valid");
        return PD_EHIP;
      }
      return PD_OK;
    }
  }
  const size_t nbar = p->nbar, ell = p->ell;
  double *zu = nullptr, *zf = nullptr;
  if (hipMalloc(&zu, nbar * sizeof(double)) != hipSuccess ||
      hipMalloc(&zf, nbar * ell * sizeof(double)) != hipSuccess) {
    if (zu) (void)hipFree(zu);
    pd_set_error("autotune: device allocation failed");
    return PD_ENOMEM;
  }
  pd_status st = PD_OK;
  if (hipMemset(zu, 0, nbar * sizeof(double)) != hipSuccess ||
      hipMemset(zf, 0, nbar * ell * sizeof(double)) != hipSuccess)
    st = PD_EHIP;
  int bestC = p->fft_C, bestMR = p->tri.MR;
  if (st == PD_OK) {
    float best = -1.f;
    for (int C = 1; C <= 32; C *= 2) {
      if (!fft_C_ok(p, C, max_lds)) continue;
      p->fft_C = C;
      const float ms =
          time_launches(p, [&] { (void)pd_launch_fft_forward(p, zu, zf, nullptr, p->spec, 0); });
      if (ms > 0.f && (best < 0.f || ms < best)) {
        best = ms;
        bestC = C;
      }
    }
    p->fft_C = bestC;
    // the spectrum now holds zeros: time the shifted solves of pass B on it
    best = -1.f;
    for (int MR : {4, 8, 16}) {
      if (!set_tri(p, MR, cus, max_lds)) continue;
      const float ms = time_launches(p, [&] {
        (void)pd_launch_tridiag(p, 0, p->spec, nullptr, nullptr);
        (void)pd_launch_reduce_partials(p, nullptr, p->bvec);
      });
      if (ms > 0.f && (best < 0.f || ms < best)) {
        best = ms;
        bestMR = MR;
      }
    }
    if (!set_tri(p, bestMR, cus, max_lds)) st = PD_EHIP;
  }
  (void)hipGetLastError();
  (void)hipFree(zu);
  (void)hipFree(zf);
  if (st != PD_OK) {
    pd_set_error("autotune: HIP error while timing candidates");
    return st;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = {bestC, bestMR};
  return PD_OK;
}

}  // namespace

extern "C" const char *paradiag_last_error(void) { return g_last_error.c_str(); }

extern "C" void paradiag_default_options(pd_options *opt) {
  if (!opt) return;
  opt->dims = 1;
  opt->precision = PD_FP64;
  opt->alpha = 1.0;
  opt->maxit = 64;
  opt->max_sweeps = 16;
  opt->check_residual = 0;
  opt->stream = nullptr;
  opt->autotune = 0;
  opt->early_exit = 0;
  opt->shifted_solver = PD_SHIFTED_PARTITION;
  opt->krylov = PD_KRYLOV_GMRES;
  opt->fom_q = 1;
  opt->bdf_order = 1;
}

extern "C" pd_status paradiag_plan_create(pd_plan *out, int n, int ell, double tau,
                                          const pd_tridiag *M, const pd_tridiag *K,
                                          const pd_options *opt_in) {
  PdRange whole("paradiag_plan_create");
  g_last_error.clear();
  if (!out) {
    pd_set_error("out is NULL");
    return PD_EINVAL;
  }
  *out = nullptr;
  pd_options opt;
  paradiag_default_options(&opt);
  if (opt_in) opt = *opt_in;
  {
    std::string msg;
    const pd_status vst = pdcheck::check_plan_args(n, ell, tau, M, K, opt, &msg);
    if (vst != PD_OK) {
      pd_set_error(msg);
      return vst;
    }
  }

  pd_plan p = new (std::nothrow) pd_plan_s();
  if (!p) {
    pd_set_error("out of host memory");
    return PD_ENOMEM;
  }
  p->n = n;
  p->ell = ell;
  p->dims = opt.dims;
  p->nbar = (opt.dims == 2) ? n * n : n;
  p->F2 = ell / 2 + 1;
  p->tau = tau;
  p->alpha = opt.alpha;
  p->w = std::pow(opt.alpha, 1.0 / ell);
  p->prec = opt.precision;
  p->maxit = opt.maxit;
  p->max_sweeps = opt.max_sweeps;
  p->check_residual = opt.check_residual;
  p->autotune = (opt.autotune != 0 && opt.dims == 1) ? 1 : 0;
  p->early_exit = opt.early_exit != 0 ? 1 : 0;
  p->sine = opt.shifted_solver == PD_SHIFTED_SINE ? 1 : 0;
  p->krylov = opt.krylov;
  p->fom_q = opt.fom_q;
  p->stream = reinterpret_cast<hipStream_t>(opt.stream);
  p->mass_identity = (M == nullptr);
  p->bdf_s = opt.bdf_order;
  bdf_coefficients(p->bdf_s, &p->bdf_beta, p->bdf_alpha);
  p->ncap = p->bdf_s * p->nbar;
  if (hipGetDevice(&p->device) != hipSuccess) {
    pd_set_error("no HIP device");
    free_plan(p);
    return PD_EHIP;
  }
  std::unique_lock<std::mutex> attr_lock(g_attr_mu);
  if (g_attr_device != p->device) {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) !=
        hipSuccess) {
      pd_set_error("hipDeviceGetAttribute failed");
      free_plan(p);
      return PD_EHIP;
    }
    g_max_lds = (size_t)lds;
    pd_fft_set_attributes(g_max_lds);
    pd_tri_set_attributes(g_max_lds);
    pd_line2d_set_attributes(g_max_lds);
    pd_fft_batch_set_attributes(g_max_lds);
    pd_tri_batch_set_attributes(g_max_lds);
    pd_sine_set_attributes(g_max_lds);
    pd_cp_set_attributes(g_max_lds);
    g_attr_device = p->device;
  }
  const size_t max_lds = g_max_lds;
  attr_lock.unlock();

  // coefficients: ML MD MU (M or I), tau*K (BDF: tau beta K, Section 5)
  const double tk = tau * p->bdf_beta;
  std::vector<double> coef(6 * (size_t)n, 0.0);
  for (int i = 0; i < n; ++i) {
    coef[i] = (M && i > 0) ? M->lower[i] : 0.0;
    coef[n + i] = M ? M->diag[i] : 1.0;
    coef[2 * n + i] = (M && i < n - 1) ? M->upper[i] : 0.0;
    coef[3 * n + i] = (i > 0) ? tk * K->lower[i] : 0.0;
    coef[4 * n + i] = tk * K->diag[i];
    coef[5 * n + i] = (i < n - 1) ? tk * K->upper[i] : 0.0;
  }
  std::vector<float> coef32(coef.begin(), coef.end());
  // Error bound factor.  With M symmetric positive definite and K symmetric
  // positive semi-definite, the scaled step (I + tau M^-1/2 K M^-1/2)^-1 has
  // norm at most 1, so the error E of any U solves a block-bidiagonal system
  // whose solution obeys ||M^1/2 E_j|| <= sum_{i<=j} ||M^-1/2 R_i||, hence
  // ||M^1/2 E||_F <= sqrt(ell (ell + 1) / 2) ||M^-1/2 R||_F; relative to
  // ||M^1/2 U||_F >= ||M U||_F / sqrt(lmax(M)) that is the factor below
  // times ||R||_F / ||M U||_F.  Symmetry is checked exactly and the
  // eigenvalue bounds by Gershgorin's theorem (backward Euler only; in 2D
  // with M = I, where K's Kronecker sum inherits the 1D bound).
  if (p->bdf_s == 1 && (p->dims == 1 || M == nullptr)) {
    bool sym = true;
    double mlo = HUGE_VAL, mhi = 0.0, klo = HUGE_VAL, kmax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double ml = coef[i], md = coef[n + i], mu = coef[2 * n + i];
      const double kl = coef[3 * n + i], kd = coef[4 * n + i], ku = coef[5 * n + i];
      if (i + 1 < n) sym = sym && coef[2 * n + i] == coef[i + 1] && coef[5 * n + i] == coef[3 * n + i + 1];
      mlo = std::min(mlo, md - std::fabs(ml) - std::fabs(mu));
      mhi = std::max(mhi, md + std::fabs(ml) + std::fabs(mu));
      klo = std::min(klo, kd - std::fabs(kl) - std::fabs(ku));
      kmax = std::max(kmax, std::fabs(kd));
    }
    if (sym && mlo > 0.0 && klo >= -1e-12 * kmax)
      p->err_factor = std::sqrt(0.5 * (double)ell * (double)(ell + 1)) * std::sqrt(mhi / mlo);
  }
  // constant diagonals (uniform grids): the shifted solves use six scalars
  {
    bool uni = true;
    const int rows_of[6][2] = {{1, n}, {0, n}, {0, n - 1}, {1, n}, {0, n}, {0, n - 1}};
    for (int d = 0; d < 6 && uni; ++d) {
      const double ref = coef[(size_t)d * n + rows_of[d][0]];
      for (int i = rows_of[d][0]; i < rows_of[d][1]; ++i)
        if (coef[(size_t)d * n + i] != ref) { uni = false; break; }
      p->uni[d] = ref;
    }
    p->uniform = uni;
  }

  // circulant constants, k = 0..ell/2
  const int F2 = p->F2;
  p->lam.assign(2 * F2, 0.0);
  p->gB.assign(2 * F2, 0.0);
  p->gJ.assign(2 * F2, 0.0);
  for (int k = 0; k < F2; ++k) {
    double c, s;
    cis(k, ell, c, s);                       // exp(+2 pi i k/ell)
    const double pr = p->w * c, pim = -p->w * s;   // pi_k = w exp(-2 pi i k/ell)
    p->lam[2 * k] = 1.0 - pr;
    p->lam[2 * k + 1] = -pim;
    const double weight = (k == 0 || 2 * k == ell) ? 1.0 : 2.0;
    const double gr = c / ell, gi = -s / ell;      // gamma_k = exp(-2 pi i k/ell)/ell
    p->gB[2 * k] = weight * gr;
    p->gB[2 * k + 1] = weight * gi;
    p->gJ[2 * k] = p->w * weight * gr;
    p->gJ[2 * k + 1] = p->w * weight * gi;
    if (p->bdf_s > 1) {
      // pi_k = sum_j alpha_j exp(-2 pi i j k / ell), the eigenvalues of C_s
      // (Section 5); pi_0 = sum_j alpha_j = 1 exactly (consistency)
      double sr = 0.0, si = 0.0;
      for (int j = 1; j <= p->bdf_s; ++j) {
        double cj, sj;
        cis((long)j * k, ell, cj, sj);
        sr += p->bdf_alpha[j - 1] * cj;
        si -= p->bdf_alpha[j - 1] * sj;
      }
      p->lam[2 * k] = (k == 0) ? 0.0 : 1.0 - sr;
      p->lam[2 * k + 1] = (k == 0 || 2 * k == ell) ? 0.0 : -si;
    }
  }
  std::vector<float> lam32(p->lam.begin(), p->lam.end());
  std::vector<double> tw(2 * (size_t)ell);
  for (int m = 0; m < ell; ++m) {
    double c, s;
    cis(m, ell, c, s);
    tw[2 * m] = c;
    tw[2 * m + 1] = -s;
  }
  std::vector<float> tw32(tw.begin(), tw.end());
  std::vector<double> dal(2 * (size_t)ell);
  for (int t = 0; t < ell; ++t) {
    dal[t] = (opt.alpha == 1.0) ? 1.0 : std::pow(opt.alpha, (double)t / ell);
    dal[ell + t] = (opt.alpha == 1.0) ? 1.0 : std::pow(opt.alpha, -(double)t / ell);
  }

  // launch configurations and sizes
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
  Layout L;
  {
    pd_status lst = compute_layout(p, cus, max_lds, L);
    if (lst != PD_OK) {
      free_plan(p);
      return lst;
    }
  }
  if (p->krylov == PD_KRYLOV_FOM && !p->sine && !pd_fom_supported(p)) {
    pd_set_error("Algorithm 2 runs on float64 plans with constant-diagonal M and K (1D: n <= "
                 "8192; the block Galerkin method: 1D)");
    free_plan(p);
    return PD_ENOTSUP;
  }
  std::vector<double> fac;
  std::vector<double> twd;
  if (p->dims == 2) {
    pd_line2d_factors(p, fac);
    const int N = p->dst_L ? p->dst_L : 2 * (n + 1);
    twd.assign(p->twd_cos + (size_t)n, 0.0);
    for (int m = 0; m < N; ++m) {
      double c, s;
      cis(m, N, c, s);
      twd[2 * m] = c;
      twd[2 * m + 1] = -s;
    }
    if (p->dst_L) chirp_tables(n, p->dst_L, &twd[p->twd_chirp], &twd[p->twd_bhat]);
    for (int j = 0; j < n; ++j) {
      double c, s;
      cis(j + 1, 2 * (n + 1), c, s);
      twd[p->twd_cos + j] = c;
    }
  } else if (p->uniform) {
    pd_uniform_factors(p, p->tri.MR, fac);
  }
  std::vector<float> fac32(fac.begin(), fac.end());
  std::vector<double> sq, swN, stwH, sm, sk;
  if (p->sine && p->dst_L) {
    twd.assign(p->twd_cos, 0.0);
    for (int m = 0; m < p->dst_L; ++m) {
      double c, s;
      cis(m, p->dst_L, c, s);
      twd[2 * m] = c;
      twd[2 * m + 1] = -s;
    }
    chirp_tables(n, p->dst_L, &twd[p->twd_chirp], &twd[p->twd_bhat]);
  }
  if (p->sine) {
    const int N = n + 1, H = N / 2;
    sq.resize(N);
    for (int j = 0; j < N; ++j) {
      double c, s;
      cis(j, 2 * (long)N, c, s);
      sq[j] = s;                              // sin(pi j / N)
    }
    swN.resize(2 * (size_t)(H + 1));
    for (int m = 0; m <= H; ++m) {
      double c, s;
      cis(m, N, c, s);
      swN[2 * m] = c;
      swN[2 * m + 1] = -s;                    // exp(-2 pi i m / N)
    }
    stwH.resize(2 * (size_t)H);
    for (int m = 0; m < H; ++m) {
      double c, s;
      cis(m, H, c, s);
      stwH[2 * m] = c;
      stwH[2 * m + 1] = -s;
    }
    sm.resize(n);
    sk.resize(n);
    for (int k = 0; k < n; ++k) {
      double c, s;
      cis(k + 1, 2 * (long)N, c, s);          // cos(pi (k+1) / N)
      sm[k] = p->uni[1] + 2.0 * p->uni[2] * c;
      sk[k] = p->uni[4] + 2.0 * p->uni[5] * c;
    }
  }
  // block Galerkin (BDF, krylov = FOM): weight_i gamma_i^(k) theta_i^(h),
  // weight_i gamma_i^(k) and theta_i^(h) for i = 0..ell/2 (Section 5), with
  // gamma^(k) = F^{-T}[e_{ell-s+1}..e_ell] A_s^T e_k, theta^(h) = F e_h
  // (the second also weights the BDF capacitance product's frequency sums)
  std::vector<double> bg_ct, bg_gt, bg_tt;
  if (p->bdf_s > 1) {
    const int s = p->bdf_s;
    bg_ct.assign(2 * (size_t)s * s * F2, 0.0);
    bg_gt.assign(2 * (size_t)s * F2, 0.0);
    bg_tt.assign(2 * (size_t)s * F2, 0.0);
    for (int i = 0; i < F2; ++i) {
      const double wgt = (i == 0 || 2 * i == ell) ? 1.0 : 2.0;
      double th[6][2], ga[6][2];
      for (int h = 0; h < s; ++h) {
        double c, sn;
        cis((long)i * h, ell, c, sn);
        th[h][0] = c;
        th[h][1] = -sn;                                // exp(-2 pi i i h / ell)
      }
      for (int k = 0; k < s; ++k) {
        double gr = 0.0, gi = 0.0;
        for (int c = k; c < s; ++c) {
          const double a = p->bdf_alpha[s - c + k - 1];   // (A_s)_{k,c}
          double cc, sn;
          cis((long)i * (ell - s + c), ell, cc, sn);       // exp(+2 pi i i (ell-s+c) / ell)
          gr += a * cc;
          gi += a * sn;
        }
        ga[k][0] = gr / ell;
        ga[k][1] = gi / ell;
      }
      for (int h = 0; h < s; ++h) {
        bg_tt[2 * ((size_t)h * F2 + i)] = th[h][0];
        bg_tt[2 * ((size_t)h * F2 + i) + 1] = th[h][1];
      }
      for (int k = 0; k < s; ++k) {
        bg_gt[2 * ((size_t)k * F2 + i)] = wgt * ga[k][0];
        bg_gt[2 * ((size_t)k * F2 + i) + 1] = wgt * ga[k][1];
        for (int h = 0; h < s; ++h) {
          const size_t q = (size_t)(k * s + h) * F2 + i;
          bg_ct[2 * q] = wgt * (ga[k][0] * th[h][0] - ga[k][1] * th[h][1]);
          bg_ct[2 * q + 1] = wgt * (ga[k][0] * th[h][1] + ga[k][1] * th[h][0]);
        }
      }
    }
  }
  std::vector<double> cptab;
  if (p->cp_on) pd_cp_tables(p, cptab);
  const size_t nbar = p->nbar;
  p->spec_bytes = L.spec_bytes;
  p->bytes = L.total_bytes();
  pd_status st = PD_OK;
#define PD_TRY(x)      \
  do {                 \
    st = (x);          \
    if (st != PD_OK) { \
      free_plan(p);    \
      return st;       \
    }                  \
  } while (0)
  PD_TRY(dev_alloc(&p->coef64, coef.size()));
  PD_TRY(dev_alloc(&p->coef32, coef32.size()));
  PD_TRY(dev_alloc(&p->lam64, p->lam.size()));
  PD_TRY(dev_alloc(&p->lam32, lam32.size()));
  PD_TRY(dev_alloc(&p->gB64, p->gB.size()));
  PD_TRY(dev_alloc(&p->gJ64, p->gJ.size()));
  PD_TRY(dev_alloc(&p->tw64, tw.size()));
  PD_TRY(dev_alloc(&p->tw32, tw32.size()));
  PD_TRY(dev_alloc(&p->dal, dal.size()));
  PD_TRY(dev_alloc(&p->fac64, std::max(fac.size(), L.fac)));
  PD_TRY(dev_alloc(&p->fac32, std::max(fac32.size(), L.fac)));
  PD_TRY(dev_alloc(&p->twd, twd.size()));
  if (p->dims == 2 || p->bdf_s > 1) PD_TRY(dev_alloc(&p->wreal, (size_t)ell * nbar));
  if (p->bdf_s > 1) {
    PD_TRY(dev_alloc(&p->wz, L.wz));
    PD_TRY(dev_alloc(&p->bdf_g, L.bdfg));
    if (p->dims == 2) {
      PD_TRY(dev_alloc(&p->bdf_h, L.bdfh));
      PD_TRY(dev_alloc(&p->bdf_t, L.bdft));
    }
  }
  PD_TRY(dev_alloc(reinterpret_cast<unsigned char **>(&p->spec), p->spec_bytes));
  if (L.spec2_bytes)
    PD_TRY(dev_alloc(reinterpret_cast<unsigned char **>(&p->spec2), L.spec2_bytes));
  PD_TRY(dev_alloc(&p->partials, L.partials));
  PD_TRY(dev_alloc(&p->rstage, L.rstage));
  PD_TRY(dev_alloc(&p->bvec, L.vec));
  PD_TRY(dev_alloc(&p->xvec, L.vec));
  PD_TRY(dev_alloc(&p->wvec, L.vec));
  PD_TRY(dev_alloc(&p->V, L.V));
  PD_TRY(dev_alloc(&p->gm, pd_gmres_state_doubles(p->maxit)));
  PD_TRY(dev_alloc(&p->red, L.red));
  if (p->cp_on) PD_TRY(dev_alloc(&p->cp_tab, L.cp));
  if (p->krylov == PD_KRYLOV_FOM) {
    PD_TRY(dev_alloc(&p->fom, L.fom));
    PD_TRY(dev_alloc(reinterpret_cast<unsigned char **>(&p->fom_h), L.fom_h_bytes));
  }
  if (p->sine) {
    PD_TRY(dev_alloc(&p->sine_q, sq.size()));
    PD_TRY(dev_alloc(&p->sine_wN, swN.size()));
    PD_TRY(dev_alloc(&p->sine_twH, stwH.size()));
    PD_TRY(dev_alloc(&p->sine_m, sm.size()));
    PD_TRY(dev_alloc(&p->sine_k, sk.size()));
  }
  // small status block written by kernels straight into pinned host memory
  if (hipHostMalloc(reinterpret_cast<void **>(&p->host_pin), 8 * sizeof(double),
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void **>(&p->host_dev), p->host_pin, 0) !=
          hipSuccess) {
    (void)hipGetLastError();
    if (p->host_pin) (void)hipHostFree(p->host_pin);
    p->host_pin = nullptr;
    pd_set_error("pinned host allocation failed");
    free_plan(p);
    return PD_ENOMEM;
  }
  PD_TRY(upload(p->coef64, coef, p->stream));
  PD_TRY(upload(p->coef32, coef32, p->stream));
  PD_TRY(upload(p->lam64, p->lam, p->stream));
  PD_TRY(upload(p->lam32, lam32, p->stream));
  PD_TRY(upload(p->gB64, p->gB, p->stream));
  PD_TRY(upload(p->gJ64, p->gJ, p->stream));
  PD_TRY(upload(p->tw64, tw, p->stream));
  PD_TRY(upload(p->tw32, tw32, p->stream));
  PD_TRY(upload(p->dal, dal, p->stream));
  PD_TRY(upload(p->fac64, fac, p->stream));
  PD_TRY(upload(p->fac32, fac32, p->stream));
  PD_TRY(upload(p->twd, twd, p->stream));
  if (p->cp_on) PD_TRY(upload(p->cp_tab, cptab, p->stream));
  if (p->bdf_s > 1) PD_TRY(upload(p->bdf_g, bg_gt, p->stream));
  if (p->krylov == PD_KRYLOV_FOM) {
    std::vector<double> mf;
    pd_fom_mass_factors(p, mf);
    const size_t mfo = p->bdf_s > 1 ? pd_bgal_layout(p->nbar, p->F2).mfac
                                    : pd_fom_mfac_offset(p->F2);
    PD_HIP_CHECK(hipMemcpyAsync(p->fom + mfo, mf.data(), mf.size() * sizeof(double),
                                hipMemcpyHostToDevice, p->stream));
    if (p->bdf_s > 1) {
      const BgLayout bl = pd_bgal_layout(p->nbar, p->F2);
      PD_HIP_CHECK(hipMemcpyAsync(p->fom + bl.ctab, bg_ct.data(), bg_ct.size() * sizeof(double),
                                  hipMemcpyHostToDevice, p->stream));
      PD_HIP_CHECK(hipMemcpyAsync(p->fom + bl.gtab, bg_gt.data(), bg_gt.size() * sizeof(double),
                                  hipMemcpyHostToDevice, p->stream));
      PD_HIP_CHECK(hipMemcpyAsync(p->fom + bl.thtab, bg_tt.data(),
                                  bg_tt.size() * sizeof(double), hipMemcpyHostToDevice,
                                  p->stream));
    }
  }
  if (p->sine) {
    PD_TRY(upload(p->sine_q, sq, p->stream));
    PD_TRY(upload(p->sine_wN, swN, p->stream));
    PD_TRY(upload(p->sine_twH, stwH, p->stream));
    PD_TRY(upload(p->sine_m, sm, p->stream));
    PD_TRY(upload(p->sine_k, sk, p->stream));
  }
#undef PD_TRY
  if (hipStreamSynchronize(p->stream) != hipSuccess) {
    pd_set_error("stream synchronisation failed during plan creation");
    free_plan(p);
    return PD_EHIP;
  }
  if (p->autotune) {
    const pd_status ts = autotune(p, cus, max_lds);
    if (ts != PD_OK) {
      free_plan(p);
      return ts;
    }
  }
  *out = p;
  return PD_OK;
}

extern "C" pd_status paradiag_plan_check(int n, int ell, double tau, const pd_tridiag *M,
                                         const pd_tridiag *K, const pd_options *opt_in) {
  g_last_error.clear();
  pd_options opt;
  paradiag_default_options(&opt);
  if (opt_in) opt = *opt_in;
  std::string msg;
  const pd_status st = pdcheck::check_plan_args(n, ell, tau, M, K, opt, &msg);
  if (st != PD_OK) pd_set_error(msg);
  return st;
}

extern "C" pd_status paradiag_plan_config(pd_plan p, int *fft_C, int *rows_per_thread) {
  if (!p) {
    pd_set_error("plan is NULL");
    return PD_EINVAL;
  }
  if (fft_C) *fft_C = p->dims == 1 ? p->fft_C : p->dst_C;
  if (rows_per_thread) *rows_per_thread = p->dims == 1 ? p->tri.MR : p->l2d.MR;
  return PD_OK;
}

extern "C" pd_status paradiag_plan_destroy(pd_plan p) {
  if (!p) {
    pd_set_error("plan is NULL");
    return PD_EINVAL;
  }
  (void)hipStreamSynchronize(p->stream);
  pd_batch_forget(p);
  free_plan(p);
  return PD_OK;
}

extern "C" size_t paradiag_spectrum_bytes(pd_plan p) { return p ? p->spec_bytes : 0; }

extern "C" size_t paradiag_plan_bytes(int n, int ell, const pd_options *opt_in) {
  pd_options opt;
  paradiag_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (n < 2 || ell < 2 || !is_pow2(ell) || ell > 4096 || opt.maxit < 1 || opt.maxit > 64 ||
      (opt.dims != 1 && opt.dims != 2))
    return 0;
  pd_plan_s tmp;
  tmp.n = n;
  tmp.ell = ell;
  tmp.dims = opt.dims;
  tmp.nbar = (opt.dims == 2) ? n * n : n;
  tmp.F2 = ell / 2 + 1;
  tmp.prec = opt.precision;
  tmp.maxit = opt.maxit;
  tmp.uniform = true;
  tmp.autotune = (opt.autotune != 0 && opt.dims == 1) ? 1 : 0;
  tmp.sine = opt.shifted_solver == PD_SHIFTED_SINE ? 1 : 0;
  tmp.krylov = opt.krylov;
  tmp.bdf_s = (opt.bdf_order >= 1 && opt.bdf_order <= 6) ? opt.bdf_order : 1;
  tmp.ncap = tmp.bdf_s * tmp.nbar;
  int dev = 0, cus = 256, lds = 65536;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  Layout L;
  if (compute_layout(&tmp, cus, (size_t)lds, L) != PD_OK) return 0;
  return L.total_bytes();
}
