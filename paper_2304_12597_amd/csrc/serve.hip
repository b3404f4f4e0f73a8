// Serving runtime: continuous batching of independent ParaDiag solves.
//
// Worker threads, each with its own HIP stream, take requests from a FIFO
// queue as soon as the device memory they account for fits the budget, so
// requests that arrive while others are running start immediately and their
// kernels overlap on the GPU.  Plans (constants, elimination factors,
// spectrum, Krylov basis) are cached per problem and reused; idle cached
// plans are evicted (least recently used first) when an admission needs the
// room.  Results do not depend on the mix: a request always runs with the
// plan configuration its own (n, ell, precision) selects, and every kernel
// reduces in a fixed order.
#include "pd_internal.h"

#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace {

struct Key {
  int n, ell, dims, prec, maxit, max_sweeps;
  // every other option a plan is built with (all but the stream)
  int check_residual, autotune, early_exit, shifted_solver, krylov, fom_q, bdf_order;
  double tau, alpha;
  std::vector<double> m, k;   // M (empty = identity) and K, row-major triples
  bool operator<(const Key &o) const {
    if (n != o.n) return n < o.n;
    if (ell != o.ell) return ell < o.ell;
    if (dims != o.dims) return dims < o.dims;
    if (prec != o.prec) return prec < o.prec;
    if (maxit != o.maxit) return maxit < o.maxit;
    if (max_sweeps != o.max_sweeps) return max_sweeps < o.max_sweeps;
    const int a[7] = {check_residual, autotune, early_exit, shifted_solver, krylov, fom_q,
                      bdf_order};
    const int b[7] = {o.check_residual, o.autotune, o.early_exit, o.shifted_solver, o.krylov,
                      o.fom_q, o.bdf_order};
    for (int q = 0; q < 7; ++q)
      if (a[q] != b[q]) return a[q] < b[q];
    if (tau != o.tau) return tau < o.tau;
    if (alpha != o.alpha) return alpha < o.alpha;
    if (m != o.m) return m < o.m;
    return k < o.k;
  }
};

struct Cached {
  pd_plan plan = nullptr;
  size_t bytes = 0;
  bool busy = false;
  unsigned long last_used = 0;
};

struct Job {
  pd_request req;
  Key key;
  std::vector<double> mcopy, kcopy;   // backing store for req.M / req.K
  pd_tridiag M, K;
  long ticket = 0;
  size_t io_bytes = 0;
  size_t plan_bytes = 0;
  bool done = false;
  pd_status status = PD_OK;
  pd_info info{};
};

std::vector<double> flatten(const pd_tridiag *t, int n) {
  std::vector<double> v;
  if (!t) return v;
  v.resize(3 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    v[3 * i] = (i > 0) ? t->lower[i] : 0.0;
    v[3 * i + 1] = t->diag[i];
    v[3 * i + 2] = (i < n - 1) ? t->upper[i] : 0.0;
  }
  return v;
}

}  // namespace

struct pd_server_s {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Job>> queue;
  std::map<long, std::shared_ptr<Job>> jobs;
  std::multimap<Key, Cached> cache;
  size_t used = 0, peak = 0;
  long next_ticket = 0, completed = 0, hits = 0, misses = 0;
  unsigned long clock = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;

  // Evict idle cached plans (LRU) until `need` more bytes fit; call locked.
  bool make_room(size_t need) {
    while (used + need > budget) {
      auto victim = cache.end();
      for (auto it = cache.begin(); it != cache.end(); ++it)
        if (!it->second.busy && (victim == cache.end() ||
                                 it->second.last_used < victim->second.last_used))
          victim = it;
      if (victim == cache.end()) return false;
      used -= victim->second.bytes;
      (void)paradiag_plan_destroy(victim->second.plan);
      cache.erase(victim);
    }
    return true;
  }

  void worker(int wid) {
    (void)hipSetDevice(device);
    hipStream_t stream = streams[wid];
    for (;;) {
      std::shared_ptr<Job> job;
      std::multimap<Key, Cached>::iterator slot = cache.end();
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stop && queue.empty()) return;
          if (!queue.empty()) {
            auto &head = queue.front();
            // an idle cached plan for this problem?
            auto range = cache.equal_range(head->key);
            for (auto it = range.first; it != range.second; ++it)
              if (!it->second.busy) { slot = it; break; }
            size_t need = head->io_bytes + (slot == cache.end() ? head->plan_bytes : 0);
            bool fits = used + need <= budget;
            if (!fits && make_room(need)) {
              fits = true;
              // eviction may have removed the slot we found
              slot = cache.end();
              auto r2 = cache.equal_range(head->key);
              for (auto it = r2.first; it != r2.second; ++it)
                if (!it->second.busy) { slot = it; break; }
              need = head->io_bytes + (slot == cache.end() ? head->plan_bytes : 0);
              fits = used + need <= budget;
            }
            if (fits) {
              job = head;
              queue.pop_front();
              used += need;
              if (used > peak) peak = used;
              if (slot != cache.end()) {
                slot->second.busy = true;
                ++hits;
              } else {
                ++misses;
              }
              break;
            }
          }
          cv_work.wait(lk);
        }
      }
      pd_plan plan = nullptr;
      pd_status st = PD_OK;
      if (slot != cache.end()) {
        plan = slot->second.plan;
      } else {
        pd_options opt = job->req.opt;
        opt.stream = stream;
        st = paradiag_plan_create(&plan, job->req.n, job->req.ell, job->req.tau,
                                  job->req.M ? &job->M : nullptr, &job->K, &opt);
      }
      if (st == PD_OK) {
        plan->stream = stream;
        st = paradiag_solve(plan, job->req.u0, job->req.F, job->req.U, job->req.tol, &job->info);
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        used -= job->io_bytes;
        if (slot != cache.end()) {
          slot->second.busy = false;
          slot->second.last_used = ++clock;
        } else if (plan) {
          Cached c;
          c.plan = plan;
          c.bytes = job->plan_bytes;
          c.last_used = ++clock;
          cache.emplace(job->key, c);
        } else {
          used -= job->plan_bytes;   // creation failed: release the reservation
        }
        job->status = st;
        job->done = true;
        ++completed;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" pd_status pd_server_create(pd_server *out, int workers, size_t budget_bytes) {
  if (!out || workers < 1 || workers > 64 || budget_bytes == 0) {
    pd_set_error("pd_server_create: invalid arguments");
    return PD_EINVAL;
  }
  *out = nullptr;
  pd_server s = new (std::nothrow) pd_server_s();
  if (!s) return PD_ENOMEM;
  s->budget = budget_bytes;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    pd_set_error("no HIP device");
    return PD_EHIP;
  }
  for (int i = 0; i < workers; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      pd_set_error("hipStreamCreate failed");
      return PD_EHIP;
    }
    s->streams.push_back(st);
  }
  for (int i = 0; i < workers; ++i) s->workers.emplace_back([s, i] { s->worker(i); });
  *out = s;
  return PD_OK;
}

extern "C" pd_status pd_server_submit(pd_server s, const pd_request *req, long *ticket) {
  if (!s || !req || !ticket || !req->K || !req->u0 || !req->F || !req->U) {
    pd_set_error("pd_server_submit: invalid arguments");
    return PD_EINVAL;
  }
  if (req->n < 2 || req->ell < 2 || req->n > 16384 || req->ell > 4096) {
    pd_set_error("pd_server_submit: sizes out of range");
    return PD_EINVAL;
  }
  auto job = std::make_shared<Job>();
  job->req = *req;
  job->mcopy = flatten(req->M, req->n);
  job->kcopy = flatten(req->K, req->n);
  // keep host copies of M and K alive for the plan creation
  const int n = req->n;
  auto unpack = [n](const std::vector<double> &v, std::vector<double> &store, pd_tridiag &t) {
    store.assign(3 * (size_t)n, 0.0);
    for (int i = 0; i < n; ++i) {
      store[i] = v[3 * i];
      store[n + i] = v[3 * i + 1];
      store[2 * n + i] = v[3 * i + 2];
    }
    t.lower = store.data();
    t.diag = store.data() + n;
    t.upper = store.data() + 2 * n;
  };
  job->key.n = req->n;
  job->key.ell = req->ell;
  job->key.dims = req->opt.dims;
  job->key.prec = req->opt.precision;
  job->key.maxit = req->opt.maxit;
  job->key.max_sweeps = req->opt.max_sweeps;
  job->key.check_residual = req->opt.check_residual;
  job->key.autotune = req->opt.autotune;
  job->key.early_exit = req->opt.early_exit;
  job->key.shifted_solver = req->opt.shifted_solver;
  job->key.krylov = req->opt.krylov;
  job->key.fom_q = req->opt.fom_q;
  job->key.bdf_order = req->opt.bdf_order;
  job->key.tau = req->tau;
  job->key.alpha = req->opt.alpha;
  job->key.m = job->mcopy;
  job->key.k = job->kcopy;
  std::vector<double> mflat = job->mcopy, kflat = job->kcopy;
  if (req->M) unpack(mflat, job->mcopy, job->M);
  unpack(kflat, job->kcopy, job->K);
  job->req.M = req->M ? &job->M : nullptr;
  job->req.K = &job->K;
  const size_t nbar = (req->opt.dims == 2) ? (size_t)n * n : (size_t)n;
  // F and U, plus u0 (BDF: the s starting values)
  const size_t starts = req->opt.bdf_order > 1 ? (size_t)req->opt.bdf_order : 1;
  job->io_bytes = (2 * (size_t)req->ell * nbar + starts * nbar) * sizeof(double);
  job->plan_bytes = paradiag_plan_bytes(req->n, req->ell, &req->opt);
  if (job->plan_bytes == 0) {
    pd_set_error("pd_server_submit: unsupported problem");
    return PD_ENOTSUP;
  }
  if (job->io_bytes + job->plan_bytes > s->budget) {
    pd_set_error("pd_server_submit: request exceeds the device-memory budget");
    return PD_EBUDGET;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    job->ticket = s->next_ticket++;
    s->jobs[job->ticket] = job;
    s->queue.push_back(job);
    *ticket = job->ticket;
  }
  s->cv_work.notify_all();
  return PD_OK;
}

extern "C" pd_status pd_server_wait(pd_server s, long ticket, int timeout_ms, int *done,
                                    pd_status *status, pd_info *info) {
  if (!s || !done) {
    pd_set_error("pd_server_wait: invalid arguments");
    return PD_EINVAL;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) {
    pd_set_error("pd_server_wait: unknown ticket");
    return PD_EINVAL;
  }
  std::shared_ptr<Job> job = it->second;
  auto ready = [&] { return job->done; };
  if (timeout_ms < 0) s->cv_done.wait(lk, ready);
  else if (timeout_ms > 0) s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  *done = job->done ? 1 : 0;
  if (job->done) {
    if (status) *status = job->status;
    if (info) *info = job->info;
    s->jobs.erase(ticket);
  }
  return PD_OK;
}

extern "C" pd_status pd_server_stats(pd_server s, long *completed, size_t *peak_bytes,
                                     long *cache_hits, long *cache_misses, size_t *current) {
  if (!s) return PD_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (peak_bytes) *peak_bytes = s->peak;
  if (cache_hits) *cache_hits = s->hits;
  if (cache_misses) *cache_misses = s->misses;
  if (current) *current = s->used;
  return PD_OK;
}

extern "C" pd_status pd_server_destroy(pd_server s) {
  if (!s) return PD_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  for (auto &kv : s->cache) (void)paradiag_plan_destroy(kv.second.plan);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return PD_OK;
}
