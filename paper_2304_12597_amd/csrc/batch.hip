// Batched solves: many independent problems, every stage launched once for
// all of them.  Each launch maps its blocks to (problem, local block) pairs,
// so problems of different sizes share the GPU in the same kernel; the
// capacitance GMRES runs in lockstep with a per-problem convergence flag.
// The per-problem arithmetic is the single-problem kernels' own (the same
// device bodies, the same reduction order), so a problem's result does not
// depend on the rest of the batch.
#include "pd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace {

bool batchable(const pd_plan *plans, int count) {
  const pd_plan p0 = plans[0];
  for (int i = 0; i < count; ++i) {
    const pd_plan p = plans[i];
    if (!p || p->dims != 1 || !p->uniform || p->prec != p0->prec || p->prec == PD_MIXED ||
        p->tri.block != pd_tri_block_threads(p->prec) ||
        p->maxit != p0->maxit)
      return false;
    for (int j = 0; j < i; ++j)
      if (plans[j] == p) return false;
  }
  return true;
}

struct DevBuf {
  void *ptr = nullptr;
  ~DevBuf() {
    if (ptr) (void)hipFree(ptr);
  }
};

}  // namespace

pd_status pd_solve_batch_impl(const pd_plan *plans, int count, const double *const *u0,
                              const double *const *F, double *const *U, double tol,
                              pd_info *infos) {
  const pd_plan p0 = plans[0];
  const hipStream_t s = p0->stream;
  const int prec = p0->prec;
  const int MX = p0->maxit;
  const size_t cb = (prec == PD_FP64) ? 16 : 8;

  std::vector<FftJob> fj(count);
  std::vector<TriJob> tj(count);
  std::vector<VecJob> vj(count);
  std::vector<int2> fftmap, tri0map, tri1map, vmap, redmap;
  int fft_threads = 64, MR = -1;
  size_t fft_lds = 0, tri_lds = 0;
  for (int i = 0; i < count; ++i) {
    const pd_plan p = plans[i];
    if (MR < 0) MR = p->tri.MR;
    if (p->tri.MR != MR) return PD_ENOTSUP;
    FftJob &f = fj[i];
    f.N = p->ell; f.n = p->n; f.nbar = p->nbar; f.dims = 1;
    f.C = p->fft_C; f.stride = p->fft_stride; f.tau = p->tau;
    f.u0 = u0[i]; f.F = F[i]; f.U = nullptr; f.coef = p->coef64; f.dal = p->dal;
    f.tw = (prec == PD_FP64) ? (const void *)p->tw64 : (const void *)p->tw32;
    f.spec = p->spec; f.out = U[i]; f.red = p->red;
    const int tiles = (p->nbar + 2 * f.C - 1) / (2 * f.C);
    for (int b = 0; b < tiles; ++b) fftmap.push_back(make_int2(i, b));
    int need = f.C * f.N / 8;
    need = ((std::max(need, 64) + 63) / 64) * 64;
    fft_threads = std::max(fft_threads, need);
    fft_lds = std::max(fft_lds, ((size_t)f.C * f.stride + pd_tw_entries(f.N)) * cb);

    TriJob &t = tj[i];
    const int P = p->tri.P;
    const int BT = pd_tri_block_threads(prec);
    if (P > BT) return PD_ENOTSUP;
    t.n = p->n; t.F2 = p->F2; t.P = P; t.spb = BT / P;
    t.nitems = pd_tri_nitems(p->tri, p->F2);
    t.nblk = std::min(t.nitems, p->tri_G);
    t.has_mass = 0;
    t.ml = p->uni[0]; t.md = p->uni[1]; t.mu = p->uni[2];
    t.kl = p->uni[3]; t.kd = p->uni[4]; t.ku = p->uni[5];
    t.coef64 = p->coef64;
    t.lam = (prec == PD_FP64) ? (const void *)p->lam64 : (const void *)p->lam32;
    t.fac = (prec == PD_FP64) ? (const void *)p->fac64 : (const void *)p->fac32;
    t.gw = p->gB64; t.in = p->spec; t.vin = nullptr; t.xv = p->xvec; t.wscale = p->w;
    t.out = p->spec; t.partials = p->partials;
    for (int b = 0; b < t.nblk; ++b) tri0map.push_back(make_int2(i, b));
    for (int b = 0; b < t.nblk; ++b) tri1map.push_back(make_int2(i, b));
    tri_lds = std::max(tri_lds, p->tri.lds);   // batchable: the same packing as p->tri

    VecJob &v = vj[i];
    v.n = p->nbar; v.B = pd_vec_blocks(p->nbar); v.G = t.nblk;
    v.V = p->V; v.w = p->wvec; v.x = p->xvec; v.red1 = p->red;
    v.red2 = p->red + (size_t)v.B * (MX + 2); v.gm = p->gm; v.partials = p->partials;
    v.bout = p->bvec; v.b = p->bvec;
    for (int b = 0; b < v.B; ++b) vmap.push_back(make_int2(i, b));
    for (int b = 0; b < (p->nbar + 255) / 256; ++b) redmap.push_back(make_int2(i, b));
  }
  // J-product jobs: same systems, mode 2, weights gamma_J, v = V_j
  std::vector<TriJob> tjJ = tj;
  for (int i = 0; i < count; ++i) {
    tjJ[i].gw = plans[i]->gJ64;
    tjJ[i].vin = plans[i]->V;
    tjJ[i].in = nullptr;
  }

  // one device buffer for the job tables, maps, flags and status
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  size_t off = 0;
  const size_t o_fj = off; off = align(off + fj.size() * sizeof(FftJob));
  const size_t o_tj = off; off = align(off + tj.size() * sizeof(TriJob));
  const size_t o_tjJ = off; off = align(off + tjJ.size() * sizeof(TriJob));
  const size_t o_vj = off; off = align(off + vj.size() * sizeof(VecJob));
  const size_t o_fm = off; off = align(off + fftmap.size() * sizeof(int2));
  const size_t o_t0 = off; off = align(off + tri0map.size() * sizeof(int2));
  const size_t o_t1 = off; off = align(off + tri1map.size() * sizeof(int2));
  const size_t o_vm = off; off = align(off + vmap.size() * sizeof(int2));
  const size_t o_rm = off; off = align(off + redmap.size() * sizeof(int2));
  const size_t o_act = off; off = align(off + count * sizeof(int));
  const size_t o_m = off; off = align(off + count * sizeof(int));
  const size_t o_st = off; off = align(off + 4 * (size_t)count * sizeof(double));
  DevBuf buf;
  if (hipMalloc(&buf.ptr, off) != hipSuccess) {
    buf.ptr = nullptr;
    pd_set_error("batched solve: device allocation failed");
    return PD_ENOMEM;
  }
  char *base = reinterpret_cast<char *>(buf.ptr);
  std::vector<char> host(off);
  auto put = [&](size_t o, const void *src, size_t bytes) { std::memcpy(host.data() + o, src, bytes); };
  put(o_fj, fj.data(), fj.size() * sizeof(FftJob));
  put(o_tj, tj.data(), tj.size() * sizeof(TriJob));
  put(o_tjJ, tjJ.data(), tjJ.size() * sizeof(TriJob));
  put(o_vj, vj.data(), vj.size() * sizeof(VecJob));
  put(o_fm, fftmap.data(), fftmap.size() * sizeof(int2));
  put(o_t0, tri0map.data(), tri0map.size() * sizeof(int2));
  put(o_t1, tri1map.data(), tri1map.size() * sizeof(int2));
  put(o_vm, vmap.data(), vmap.size() * sizeof(int2));
  put(o_rm, redmap.data(), redmap.size() * sizeof(int2));
  PD_HIP_CHECK(hipMemcpyAsync(buf.ptr, host.data(), o_act, hipMemcpyHostToDevice, s));
  const FftJob *d_fj = reinterpret_cast<const FftJob *>(base + o_fj);
  const TriJob *d_tj = reinterpret_cast<const TriJob *>(base + o_tj);
  const TriJob *d_tjJ = reinterpret_cast<const TriJob *>(base + o_tjJ);
  const VecJob *d_vj = reinterpret_cast<const VecJob *>(base + o_vj);
  const int2 *d_fm = reinterpret_cast<const int2 *>(base + o_fm);
  const int2 *d_t0 = reinterpret_cast<const int2 *>(base + o_t0);
  const int2 *d_t1 = reinterpret_cast<const int2 *>(base + o_t1);
  const int2 *d_vm = reinterpret_cast<const int2 *>(base + o_vm);
  const int2 *d_rm = reinterpret_cast<const int2 *>(base + o_rm);
  int *d_act = reinterpret_cast<int *>(base + o_act);
  int *d_m = reinterpret_cast<int *>(base + o_m);
  double *d_st = reinterpret_cast<double *>(base + o_st);
  const int nf = (int)fftmap.size(), n0 = (int)tri0map.size(), n1 = (int)tri1map.size();
  const int nv = (int)vmap.size(), nr = (int)redmap.size();

  pd_status st;
#define PD_B(x)                    \
  do {                             \
    st = (x);                      \
    if (st != PD_OK) return st;    \
  } while (0)
  // first stage and first parfor with the b reduction
  PD_B(pd_launch_fft_forward_batch(prec, d_fj, d_fm, nf, fft_threads, fft_lds, s));
  PD_B(pd_launch_tridiag_batch(prec, MR, 0, d_tj, d_t0, n0, tri_lds, nullptr, 0, s));
  PD_B(pd_launch_reduce_batch(d_vj, d_rm, nr, -1, nullptr, s));
  // capacitance GMRES in lockstep
  PD_B(pd_gmres_batch_dots(d_vj, d_vm, nv, 0, 1, nullptr, s));
  PD_B(pd_gmres_batch_init(d_vj, count, MX, d_st, s));
  PD_B(pd_gmres_batch_scale(d_vj, d_vm, nv, 0, MX, 1, nullptr, s));
  std::vector<double> hst(4 * (size_t)count);
  PD_HIP_CHECK(hipMemcpyAsync(hst.data(), d_st, hst.size() * sizeof(double),
                              hipMemcpyDeviceToHost, s));
  PD_HIP_CHECK(hipStreamSynchronize(s));
  std::vector<int> act(count), m(count, 0);
  std::vector<double> beta(count), res(count);
  int nact = 0;
  for (int i = 0; i < count; ++i) {
    beta[i] = hst[4 * i];
    if (!std::isfinite(beta[i])) {
      pd_set_error("batched solve: non-finite capacitance right-hand side");
      return PD_ENONFINITE;
    }
    res[i] = beta[i];
    act[i] = beta[i] > 0.0;
    nact += act[i];
  }
  const double rtol = tol * PD_GMRES_TOL_FACTOR;
  // 1D problems of at most pd_gmres_fused_max_n() unknowns take the fused
  // Arnoldi step, as they do when solved alone
  bool fused = true;
  for (int i = 0; i < count; ++i) fused = fused && plans[i]->nbar <= pd_gmres_fused_max_n();
  for (int j = 0; j < MX && nact > 0; ++j) {
    PD_HIP_CHECK(hipMemcpyAsync(d_act, act.data(), count * sizeof(int), hipMemcpyHostToDevice, s));
    PD_B(pd_launch_tridiag_batch(prec, MR, 2, d_tjJ, d_t0, n0, tri_lds, d_act, j, s));
    PD_B(pd_launch_reduce_batch(d_vj, d_rm, nr, j, d_act, s));
    if (fused) {
      PD_B(pd_gmres_batch_arnoldi(d_vj, count, j, MX, rtol, d_st, d_act, s));
    } else {
      PD_B(pd_gmres_batch_dots(d_vj, d_vm, nv, j + 1, 0, d_act, s));
      PD_B(pd_gmres_batch_update(d_vj, d_vm, nv, j + 1, j, MX, 1, d_act, s));
      PD_B(pd_gmres_batch_update(d_vj, d_vm, nv, j + 1, j, MX, 2, d_act, s));
      PD_B(pd_gmres_batch_dots(d_vj, d_vm, nv, 0, 0, d_act, s));
      PD_B(pd_gmres_batch_givens(d_vj, count, j, MX, d_st, d_act, s));
      PD_B(pd_gmres_batch_scale(d_vj, d_vm, nv, j, MX, 0, d_act, s));
    }
    PD_HIP_CHECK(hipMemcpyAsync(hst.data(), d_st, hst.size() * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    PD_HIP_CHECK(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i) {
      if (!act[i]) continue;
      m[i] = j + 1;
      res[i] = hst[4 * i];
      if (!std::isfinite(res[i])) {
        pd_set_error("batched solve: non-finite GMRES residual");
        return PD_ENONFINITE;
      }
      if (res[i] <= rtol * beta[i] || hst[4 * i + 1] == 0.0) {
        act[i] = 0;
        --nact;
      }
    }
  }
  PD_HIP_CHECK(hipMemcpyAsync(d_m, m.data(), count * sizeof(int), hipMemcpyHostToDevice, s));
  PD_B(pd_gmres_batch_finish(d_vj, d_vm, nv, count, MX, d_m, s));
  // second parfor and last stage
  PD_B(pd_launch_tridiag_batch(prec, MR, 1, d_tj, d_t1, n1, tri_lds, nullptr, 0, s));
  PD_B(pd_launch_fft_inverse_batch(prec, d_fj, d_fm, nf, fft_threads, fft_lds, s));
#undef PD_B
  PD_HIP_CHECK(hipStreamSynchronize(s));
  pd_status worst = PD_OK;
  for (int i = 0; i < count; ++i) {
    const bool conv = beta[i] == 0.0 || res[i] <= rtol * beta[i];
    if (!conv) worst = PD_ENOTCONV;
    if (infos) {
      infos[i].gmres_iters = m[i];
      infos[i].sweeps = 1;
      infos[i].pint_loops = m[i] + 2;
      infos[i].gmres_rel_residual = beta[i] > 0.0 ? res[i] / beta[i] : 0.0;
      infos[i].rel_residual = -1.0;
      if (plans[i]->check_residual) {
        double rel;
        pd_status rs = pd_residual_impl(plans[i], u0[i], F[i], U[i], &rel);
        if (rs != PD_OK) return rs;
        infos[i].rel_residual = rel;
      }
    }
  }
  if (worst == PD_ENOTCONV) pd_set_error("tolerance not reached for some problems");
  return worst;
}

bool pd_batchable(const pd_plan *plans, int count) { return count > 0 && batchable(plans, count); }
