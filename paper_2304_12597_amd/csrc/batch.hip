// Batched solves: many independent problems, every stage launched once for
// all of them.  Each launch maps its blocks to (problem, local block) pairs,
// so problems of different sizes share the GPU in the same kernel; the
// capacitance GMRES runs in lockstep, each problem stopping on its own
// device-side convergence flag.  The per-problem arithmetic is the
// single-problem kernels' own (the same device bodies, the same reduction
// order), so a problem's result does not depend on the rest of the batch.
//
// The whole solve -- transforms, parfors, K GMRES iterations, x = V y --
// is one launch sequence with no host round trip; once every plan of a
// batch has been solved before (K = the largest iteration count they
// needed), the sequence is captured as a HIP graph, cached per (plans,
// arrays, tol, K) and replayed.  If some problem has not converged after K
// iterations, an uncaptured loop continues it and the tail is redone.
#include "pd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <vector>

namespace {

bool batchable(const pd_plan *plans, int count) {
  const pd_plan p0 = plans[0];
  for (int i = 0; i < count; ++i) {
    const pd_plan p = plans[i];
    if (!p || p->dims != 1 || !p->uniform || p->prec != p0->prec || p->prec == PD_MIXED ||
        p->tri.block != pd_tri_block_threads(p->prec) ||
        p->maxit != p0->maxit || p->early_exit || p->sine || p->krylov || p->bdf_s > 1 ||
        !pd_gmres_fused_ok(p))
      return false;
    for (int j = 0; j < i; ++j)
      if (plans[j] == p) return false;
  }
  return true;
}

// Device tables of one batch shape, its pinned status copy and (once the
// iteration count is known) its captured graph.
struct BatchRun {
  std::vector<const void *> key;   // plans, u0, F, U
  double tol = 0.0;
  int K = 0, count = 0, prec = 0, MX = 0;
  // shifted-solve launches, one per rows-per-thread bucket (MR 4, 8, 16):
  // each bucket's entries are contiguous in the t0, t1, t0J and k0m maps
  struct TriBucket {
    int MR = 0, o0 = 0, n0 = 0, o1 = 0, n1 = 0, o0J = 0, n0J = 0, ok0 = 0, nk0 = 0;
    size_t lds = 0;
  } tb[3];
  hipStream_t s = nullptr;
  void *dev = nullptr;
  double *pin = nullptr;           // statuses [4 * count]: residual, h, iterations, beta
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;       // capture stream (the plan stream may be the legacy one)
  const FftJob *fj = nullptr;
  const TriJob *tj = nullptr, *tjJ = nullptr, *tk0 = nullptr;
  const int2 *k0m = nullptr;
  int nk0 = 0;
  const VecJob *vj = nullptr;
  const int2 *fm = nullptr, *t0 = nullptr, *t1 = nullptr, *vm = nullptr, *rm = nullptr;
  // J products: the per-frequency path (t0J, rmJ) for some problems, the
  // chunked capacitance product (cj, c1m..c3m) for the others
  const int2 *t0J = nullptr, *rmJ = nullptr;
  const CpJob *cj = nullptr;
  const int2 *c1m = nullptr, *c2m = nullptr, *c3m = nullptr;
  int *act = nullptr;
  double *st = nullptr;
  int nf = 0, n0 = 0, n1 = 0, nv = 0, nr = 0, fft_threads = 64;
  int n0J = 0, nrJ = 0, nc1 = 0, nc2 = 0, nc3 = 0, cthreads2 = 64;
  size_t fft_lds = 0, clds1 = 0, clds2 = 0;
  ~BatchRun() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cap) (void)hipStreamDestroy(cap);
    if (dev) (void)hipFree(dev);
    if (pin) (void)hipHostFree(pin);
  }
};

std::mutex g_runs_mu;
std::list<std::unique_ptr<BatchRun>> g_runs;   // most recent first
constexpr size_t kMaxRuns = 4;

pd_status build_run(BatchRun &r, const pd_plan *plans, int count, const double *const *u0,
                    const double *const *F, double *const *U) {
  const pd_plan p0 = plans[0];
  const int prec = p0->prec;
  const int MX = p0->maxit;
  const size_t cb = (prec == PD_FP64) ? 16 : 8;
  r.count = count;
  r.prec = prec;
  r.MX = MX;
  r.s = p0->stream;
  {
    std::vector<FftJob> fj(count);
    std::vector<TriJob> tj(count);
    std::vector<VecJob> vj(count);
    std::vector<int2> fftmap, tri0map, tri1map, vmap, redmap, tri0mapJ, redmapJ;
    std::vector<CpJob> cj(count);
    std::vector<int2> c1map, c2map, c3map, k0map;
    int cthreads2 = 64;
    size_t clds1 = 0, clds2 = 0;
    int fft_threads = 64;
    size_t fft_lds = 0;
    // per rows-per-thread bucket: the shifted-solve block maps and LDS size
    std::vector<int2> t0b[3], t1b[3], t0Jb[3], k0b[3];
    size_t ldsb[3] = {0, 0, 0};
    for (int i = 0; i < count; ++i) {
      const pd_plan p = plans[i];
      const int bi = p->tri.MR == 4 ? 0 : (p->tri.MR == 8 ? 1 : 2);
      if (p->tri.MR != 4 && p->tri.MR != 8 && p->tri.MR != 16) return PD_ENOTSUP;
      FftJob &f = fj[i];
      f.N = p->ell; f.n = p->n; f.nbar = p->nbar; f.dims = 1;
      f.C = p->fft_C; f.stride = p->fft_stride; f.tau = p->tau;
      f.u0 = u0[i]; f.F = F[i]; f.U = nullptr; f.coef = p->coef64; f.dal = p->alpha == 1.0 ? nullptr : p->dal;
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
      t.scan = (prec == PD_FP64 && pd_use_scan(p)) ? 1 : 0;
      t.gw = p->gB64; t.in = p->spec; t.vin = nullptr; t.xv = p->xvec; t.wscale = p->w;
      t.out = p->spec; t.partials = p->partials; t.skip = nullptr;
      for (int b = 0; b < t.nblk; ++b) t0b[bi].push_back(make_int2(i, b));
      for (int b = 0; b < t.nblk; ++b) t1b[bi].push_back(make_int2(i, b));
      ldsb[bi] = std::max(ldsb[bi], p->tri.lds);   // batchable: the same packing as p->tri

      VecJob &v = vj[i];
      v.n = p->nbar; v.B = pd_vec_blocks(p->nbar); v.G = t.nblk;
      v.V = p->V; v.w = p->wvec; v.x = p->xvec; v.red1 = p->red;
      v.red2 = p->red + (size_t)v.B * (MX + 2); v.gm = p->gm; v.partials = p->partials;
      v.bout = p->bvec; v.b = p->bvec; v.done = p->gm + pd_gmres_done_index(MX);
      for (int b = 0; b < v.B; ++b) vmap.push_back(make_int2(i, b));
      for (int b = 0; b < (p->nbar + 255) / 256; ++b) redmap.push_back(make_int2(i, b));
      if (p->cp_on) {
        // J products of this problem by the chunked capacitance product (jobs
        // indexed by problem, like the activity flags)
        const CpJob J = pd_cp_job(p, p->V, p->wvec, p->gm + pd_gmres_done_index(MX));
        cj[i] = J;
        for (int b = 0; b < pd_cp_blocks(J, 1); ++b) c1map.push_back(make_int2(i, b));
        for (int b = 0; b < pd_cp_blocks(J, 2); ++b) c2map.push_back(make_int2(i, b));
        for (int b = 0; b < pd_cp_blocks(J, 3); ++b) c3map.push_back(make_int2(i, b));
        if (p->cpl.k0sep) k0b[bi].push_back(make_int2(i, 0));
        cthreads2 = std::max(cthreads2, pd_cp_threads2(J));
        clds1 = std::max(clds1, pd_cp_lds(J, 1));
        clds2 = std::max(clds2, pd_cp_lds(J, 2));
      } else {
        for (int b = 0; b < t.nblk; ++b) t0Jb[bi].push_back(make_int2(i, b));
        for (int b = 0; b < (p->nbar + 255) / 256; ++b) redmapJ.push_back(make_int2(i, b));
      }
    }
    for (int bi = 0; bi < 3; ++bi) {
      auto &B = r.tb[bi];
      B.MR = 4 << bi;
      B.lds = ldsb[bi];
      B.o0 = (int)tri0map.size();
      B.n0 = (int)t0b[bi].size();
      tri0map.insert(tri0map.end(), t0b[bi].begin(), t0b[bi].end());
      B.o1 = (int)tri1map.size();
      B.n1 = (int)t1b[bi].size();
      tri1map.insert(tri1map.end(), t1b[bi].begin(), t1b[bi].end());
      B.o0J = (int)tri0mapJ.size();
      B.n0J = (int)t0Jb[bi].size();
      tri0mapJ.insert(tri0mapJ.end(), t0Jb[bi].begin(), t0Jb[bi].end());
      B.ok0 = (int)k0map.size();
      B.nk0 = (int)k0b[bi].size();
      k0map.insert(k0map.end(), k0b[bi].begin(), k0b[bi].end());
    }
    // J-product jobs: same systems, mode 2, weights gamma_J, v = V_j
    std::vector<TriJob> tjJ = tj;
    for (int i = 0; i < count; ++i) {
      tjJ[i].gw = plans[i]->gJ64;
      tjJ[i].vin = plans[i]->V;
      tjJ[i].in = nullptr;
      tjJ[i].skip = plans[i]->gm + pd_gmres_done_index(MX);
    }
    // the k = 0 term of chunked-product problems that take it through the
    // shifted-solve body: one block, the first item, weights at k = 0 only
    std::vector<TriJob> tjK0 = tjJ;
    for (int i = 0; i < count; ++i)
      if (plans[i]->cp_on && plans[i]->cpl.k0sep) {
        tjK0[i].gw = plans[i]->cp_tab + plans[i]->cpl.gJ0;
        tjK0[i].nitems = 1;
        tjK0[i].nblk = 1;
      }

    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_fj = off; off = align(off + fj.size() * sizeof(FftJob));
    const size_t o_tj = off; off = align(off + tj.size() * sizeof(TriJob));
    const size_t o_tjJ = off; off = align(off + tjJ.size() * sizeof(TriJob));
    const size_t o_tk0 = off; off = align(off + tjK0.size() * sizeof(TriJob));
    const size_t o_k0 = off; off = align(off + k0map.size() * sizeof(int2));
    const size_t o_vj = off; off = align(off + vj.size() * sizeof(VecJob));
    const size_t o_fm = off; off = align(off + fftmap.size() * sizeof(int2));
    const size_t o_t0 = off; off = align(off + tri0map.size() * sizeof(int2));
    const size_t o_t1 = off; off = align(off + tri1map.size() * sizeof(int2));
    const size_t o_vm = off; off = align(off + vmap.size() * sizeof(int2));
    const size_t o_rm = off; off = align(off + redmap.size() * sizeof(int2));
    const size_t o_t0J = off; off = align(off + tri0mapJ.size() * sizeof(int2));
    const size_t o_rmJ = off; off = align(off + redmapJ.size() * sizeof(int2));
    const size_t o_cj = off; off = align(off + cj.size() * sizeof(CpJob));
    const size_t o_c1 = off; off = align(off + c1map.size() * sizeof(int2));
    const size_t o_c2 = off; off = align(off + c2map.size() * sizeof(int2));
    const size_t o_c3 = off; off = align(off + c3map.size() * sizeof(int2));
    const size_t o_act = off; off = align(off + count * sizeof(int));
    const size_t o_st = off; off = align(off + 4 * (size_t)count * sizeof(double));
    if (hipMalloc(&r.dev, off) != hipSuccess) {
      r.dev = nullptr;
      pd_set_error("batched solve: device allocation failed");
      return PD_ENOMEM;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&r.pin), 4 * (size_t)count * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
      r.pin = nullptr;
      pd_set_error("batched solve: pinned allocation failed");
      return PD_ENOMEM;
    }
    std::vector<char> host(o_act);
    auto put = [&](size_t o, const void *src, size_t bytes) {
      std::memcpy(host.data() + o, src, bytes);
    };
    put(o_fj, fj.data(), fj.size() * sizeof(FftJob));
    put(o_tj, tj.data(), tj.size() * sizeof(TriJob));
    put(o_tjJ, tjJ.data(), tjJ.size() * sizeof(TriJob));
    put(o_tk0, tjK0.data(), tjK0.size() * sizeof(TriJob));
    put(o_k0, k0map.data(), k0map.size() * sizeof(int2));
    put(o_vj, vj.data(), vj.size() * sizeof(VecJob));
    put(o_fm, fftmap.data(), fftmap.size() * sizeof(int2));
    put(o_t0, tri0map.data(), tri0map.size() * sizeof(int2));
    put(o_t1, tri1map.data(), tri1map.size() * sizeof(int2));
    put(o_vm, vmap.data(), vmap.size() * sizeof(int2));
    put(o_rm, redmap.data(), redmap.size() * sizeof(int2));
    put(o_t0J, tri0mapJ.data(), tri0mapJ.size() * sizeof(int2));
    put(o_rmJ, redmapJ.data(), redmapJ.size() * sizeof(int2));
    put(o_cj, cj.data(), cj.size() * sizeof(CpJob));
    put(o_c1, c1map.data(), c1map.size() * sizeof(int2));
    put(o_c2, c2map.data(), c2map.size() * sizeof(int2));
    put(o_c3, c3map.data(), c3map.size() * sizeof(int2));
    PD_HIP_CHECK(hipMemcpy(r.dev, host.data(), o_act, hipMemcpyHostToDevice));
    char *base = reinterpret_cast<char *>(r.dev);
    r.fj = reinterpret_cast<const FftJob *>(base + o_fj);
    r.tj = reinterpret_cast<const TriJob *>(base + o_tj);
    r.tjJ = reinterpret_cast<const TriJob *>(base + o_tjJ);
    r.tk0 = reinterpret_cast<const TriJob *>(base + o_tk0);
    r.k0m = reinterpret_cast<const int2 *>(base + o_k0);
    r.nk0 = (int)k0map.size();
    r.vj = reinterpret_cast<const VecJob *>(base + o_vj);
    r.fm = reinterpret_cast<const int2 *>(base + o_fm);
    r.t0 = reinterpret_cast<const int2 *>(base + o_t0);
    r.t1 = reinterpret_cast<const int2 *>(base + o_t1);
    r.vm = reinterpret_cast<const int2 *>(base + o_vm);
    r.rm = reinterpret_cast<const int2 *>(base + o_rm);
    r.t0J = reinterpret_cast<const int2 *>(base + o_t0J);
    r.rmJ = reinterpret_cast<const int2 *>(base + o_rmJ);
    r.cj = reinterpret_cast<const CpJob *>(base + o_cj);
    r.c1m = reinterpret_cast<const int2 *>(base + o_c1);
    r.c2m = reinterpret_cast<const int2 *>(base + o_c2);
    r.c3m = reinterpret_cast<const int2 *>(base + o_c3);
    r.n0J = (int)tri0mapJ.size();
    r.nrJ = (int)redmapJ.size();
    r.nc1 = (int)c1map.size();
    r.nc2 = (int)c2map.size();
    r.nc3 = (int)c3map.size();
    r.cthreads2 = cthreads2;
    r.clds1 = clds1;
    r.clds2 = clds2;
    r.act = reinterpret_cast<int *>(base + o_act);
    r.st = reinterpret_cast<double *>(base + o_st);
    r.nf = (int)fftmap.size();
    r.n0 = (int)tri0map.size();
    r.n1 = (int)tri1map.size();
    r.nv = (int)vmap.size();
    r.nr = (int)redmap.size();
    r.fft_threads = fft_threads;
    r.fft_lds = fft_lds;
  }
  return PD_OK;
}

#define PD_B(x)                 \
  do {                          \
    pd_status st_ = (x);        \
    if (st_ != PD_OK) return st_; \
  } while (0)

// One shifted-solve launch per rows-per-thread bucket present in the batch
// (map, off, cnt: which of the bucket's block maps).
pd_status tri_batch(const BatchRun &r, int mode, const TriJob *jobs, const int2 *map,
                    int BatchRun::TriBucket::*off, int BatchRun::TriBucket::*cnt, const int *act,
                    int j, hipStream_t s) {
  for (const auto &B : r.tb)
    if (B.*cnt > 0)
      PD_B(pd_launch_tridiag_batch(r.prec, B.MR, mode, jobs, map + B.*off, B.*cnt, B.lds, act, j,
                                   s));
  return PD_OK;
}
using TB = BatchRun::TriBucket;

// w = J V_j for every problem still iterating: the per-frequency product
// and its reduction, and the chunked capacitance product.
pd_status j_products(const BatchRun &r, int j, const int *act, hipStream_t s) {
  PD_B(tri_batch(r, 2, r.tjJ, r.t0J, &TB::o0J, &TB::n0J, act, j, s));
  PD_B(pd_launch_reduce_batch(r.vj, r.rmJ, r.nrJ, j, act, s));
  PD_B(tri_batch(r, 2, r.tk0, r.k0m, &TB::ok0, &TB::nk0, act, j, s));
  PD_B(pd_cp_launch_batch(r.cj, r.c1m, r.nc1, r.c2m, r.nc2, r.cthreads2, r.c3m, r.nc3, r.clds1,
                          r.clds2, act, j, s));
  return PD_OK;
}

// The launch sequence of one batched solve with K GMRES iterations (no
// synchronisation, no host data: capturable).
pd_status enqueue_solve(const BatchRun &r, int K, double rtol, hipStream_t s) {
  PD_B(pd_launch_fft_forward_batch(r.prec, r.fj, r.fm, r.nf, r.fft_threads, r.fft_lds, s));
  PD_B(tri_batch(r, 0, r.tj, r.t0, &TB::o0, &TB::n0, nullptr, 0, s));
  PD_B(pd_launch_reduce_batch(r.vj, r.rm, r.nr, -1, nullptr, s));
  PD_B(pd_gmres_batch_start(r.vj, r.count, r.MX, r.st, s));
  for (int j = 0; j < K; ++j) {
    PD_B(j_products(r, j, nullptr, s));
    PD_B(pd_gmres_batch_arnoldi(r.vj, r.count, j, r.MX, rtol, r.st, nullptr, s));
  }
  PD_B(pd_gmres_batch_finish(r.vj, r.vm, r.nv, r.count, r.MX, nullptr, s));
  PD_B(tri_batch(r, 1, r.tj, r.t1, &TB::o1, &TB::n1, nullptr, 0, s));
  PD_B(pd_launch_fft_inverse_batch(r.prec, r.fj, r.fm, r.nf, r.fft_threads, r.fft_lds, s));
  PD_HIP_CHECK(hipMemcpyAsync(r.pin, r.st, 4 * (size_t)r.count * sizeof(double),
                              hipMemcpyDeviceToHost, s));
  return PD_OK;
}

bool converged(const double *st, double rtol) {
  const double res = st[0], hn = st[1], beta = st[3];
  return beta == 0.0 || res <= rtol * beta || hn == 0.0;
}

// Problems still iterating after K steps (all at iteration K) continue
// with host-checked steps; then pass A is redone for every problem (pass C
// overwrote the spectra) and the tail is run again.
pd_status finish_unconverged(const BatchRun &r, int K, double rtol) {
  const hipStream_t s = r.s;
  std::vector<int> act(r.count);
  int nact = 0;
  for (int i = 0; i < r.count; ++i) {
    act[i] = !converged(r.pin + 4 * i, rtol) && (int)r.pin[4 * i + 2] < r.MX;
    nact += act[i];
  }
  if (nact == 0) return PD_OK;
  for (int j = K; j < r.MX && nact > 0; ++j) {
    PD_HIP_CHECK(hipMemcpyAsync(r.act, act.data(), r.count * sizeof(int), hipMemcpyHostToDevice, s));
    PD_B(j_products(r, j, r.act, s));
    PD_B(pd_gmres_batch_arnoldi(r.vj, r.count, j, r.MX, rtol, r.st, r.act, s));
    PD_HIP_CHECK(hipMemcpyAsync(r.pin, r.st, 4 * (size_t)r.count * sizeof(double),
                                hipMemcpyDeviceToHost, s));
    PD_HIP_CHECK(hipStreamSynchronize(s));
    for (int i = 0; i < r.count; ++i) {
      if (!act[i]) continue;
      const double *st = r.pin + 4 * i;
      if (!std::isfinite(st[0]) || converged(st, rtol)) {
        act[i] = 0;
        --nact;
      }
    }
  }
  PD_B(pd_launch_fft_forward_batch(r.prec, r.fj, r.fm, r.nf, r.fft_threads, r.fft_lds, s));
  PD_B(pd_gmres_batch_finish(r.vj, r.vm, r.nv, r.count, r.MX, nullptr, s));
  PD_B(tri_batch(r, 1, r.tj, r.t1, &TB::o1, &TB::n1, nullptr, 0, s));
  PD_B(pd_launch_fft_inverse_batch(r.prec, r.fj, r.fm, r.nf, r.fft_threads, r.fft_lds, s));
  PD_HIP_CHECK(hipStreamSynchronize(s));
  return PD_OK;
}

}  // namespace

void pd_batch_forget(pd_plan p) {
  std::lock_guard<std::mutex> lk(g_runs_mu);
  g_runs.remove_if([p](const std::unique_ptr<BatchRun> &r) {
    for (int i = 0; i < r->count; ++i)
      if (r->key[i] == p) return true;
    return false;
  });
}

pd_status pd_solve_batch_impl(const pd_plan *plans, int count, const double *const *u0,
                              const double *const *F, double *const *U, double tol,
                              pd_info *infos) {
  const pd_plan p0 = plans[0];
  const int MX = p0->maxit;
  const double rtol = pd_gmres_tol(p0->prec, tol);
  bool learned = true;
  int K = 1;
  for (int i = 0; i < count; ++i) {
    learned = learned && plans[i]->gm_seen;
    K = std::max(K, plans[i]->gm_pred);
  }
  K = std::min(K, MX);
  std::vector<const void *> key;
  key.reserve(4 * (size_t)count);
  for (int i = 0; i < count; ++i) key.push_back(plans[i]);
  for (int i = 0; i < count; ++i) key.push_back(u0[i]);
  for (int i = 0; i < count; ++i) key.push_back(F[i]);
  for (int i = 0; i < count; ++i) key.push_back(U[i]);

  std::lock_guard<std::mutex> lk(g_runs_mu);
  BatchRun *run = nullptr;
  for (auto it = g_runs.begin(); it != g_runs.end(); ++it)
    if ((*it)->key == key && (*it)->tol == tol && (*it)->K == K && (*it)->s == p0->stream) {
      g_runs.splice(g_runs.begin(), g_runs, it);   // most recent first
      run = g_runs.front().get();
      break;
    }
  if (!run) {
    auto fresh = std::make_unique<BatchRun>();
    fresh->key = key;
    fresh->tol = tol;
    fresh->K = K;
    pd_status bs = build_run(*fresh, plans, count, u0, F, U);
    if (bs != PD_OK) return bs;
    g_runs.push_front(std::move(fresh));
    if (g_runs.size() > kMaxRuns) g_runs.pop_back();
    run = g_runs.front().get();
  }
  const hipStream_t s = run->s;
  if (learned && !run->exec) {
    // capture once; replays are a single launch
    hipGraph_t graph = nullptr;
    if (!run->cap) PD_HIP_CHECK(hipStreamCreateWithFlags(&run->cap, hipStreamNonBlocking));
    PD_HIP_CHECK(hipStreamBeginCapture(run->cap, hipStreamCaptureModeThreadLocal));
    const pd_status es = enqueue_solve(*run, K, rtol, run->cap);
    const hipError_t ce = hipStreamEndCapture(run->cap, &graph);
    if (es != PD_OK || ce != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (es != PD_OK) return es;
      pd_set_error("batched solve: graph capture failed");
      return PD_EHIP;
    }
    const hipError_t ie = hipGraphInstantiate(&run->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      run->exec = nullptr;
      pd_set_error("batched solve: graph instantiation failed");
      return PD_EHIP;
    }
  }
  if (run->exec) {
    PD_HIP_CHECK(hipGraphLaunch(run->exec, s));
  } else {
    PD_B(enqueue_solve(*run, K, rtol, s));
  }
  PD_HIP_CHECK(hipStreamSynchronize(s));
  for (int i = 0; i < count; ++i) {
    if (!std::isfinite(run->pin[4 * i + 3])) {
      pd_set_error("batched solve: non-finite capacitance right-hand side");
      return PD_ENONFINITE;
    }
    if (!std::isfinite(run->pin[4 * i])) {
      pd_set_error("batched solve: non-finite GMRES residual");
      return PD_ENONFINITE;
    }
  }
  PD_B(finish_unconverged(*run, K, rtol));

  pd_status worst = PD_OK;
  for (int i = 0; i < count; ++i) {
    const double *st = run->pin + 4 * i;
    const int m = (int)st[2];
    const double res = st[0], beta = st[3];
    const bool conv = converged(st, rtol);
    if (!conv) worst = PD_ENOTCONV;
    plans[i]->gm_seen = 1;
    if (m > 0) plans[i]->gm_pred = m;
    if (infos) {
      infos[i].gmres_iters = m;
      infos[i].sweeps = 1;
      infos[i].pint_loops = m + 2;
      infos[i].gmres_rel_residual = beta > 0.0 ? res / beta : 0.0;
      infos[i].rel_residual = -1.0;
      infos[i].est_rel_error = -1.0;
      infos[i].early_exit = 0;
      if (plans[i]->check_residual) {
        double rel, est;
        pd_status rs = pd_residual_impl(plans[i], u0[i], F[i], U[i], &rel, &est);
        if (rs != PD_OK) return rs;
        infos[i].rel_residual = rel;
        infos[i].est_rel_error = est;
      }
    }
  }
  if (worst == PD_ENOTCONV) pd_set_error("tolerance not reached for some problems");
  return worst;
}
#undef PD_B

bool pd_batchable(const pd_plan *plans, int count) { return count > 0 && batchable(plans, count); }
