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
#include "pd_admission.h"
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
  using Policy = pdserve::Admission<Key, pd_plan>;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Job>> queue;
  std::map<long, std::shared_ptr<Job>> jobs;
  Policy policy;
  long next_ticket = 0, completed = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;

  explicit pd_server_s(size_t budget) : policy(budget) {}

  void worker(int wid) {
    (void)hipSetDevice(device);
    hipStream_t stream = streams[wid];
    for (;;) {
      std::shared_ptr<Job> job;
      Policy::Grant grant;
      std::vector<std::pair<Key, pd_plan>> evicted;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (stop && queue.empty()) return;
          if (!queue.empty()) {
            auto &head = queue.front();
            grant = policy.try_admit(head->key, head->io_bytes, head->plan_bytes, &evicted);
            if (grant.admitted) {
              job = head;
              queue.pop_front();
              break;
            }
          }
          cv_work.wait(lk);
        }
      }
      for (auto &e : evicted) (void)paradiag_plan_destroy(e.second);
      pd_plan plan = nullptr;
      pd_status st = PD_OK;
      if (grant.hit) {
        plan = grant.slot->second.handle;
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
        policy.finish(grant, job->key, plan != nullptr, plan);
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
  pd_server s = new (std::nothrow) pd_server_s(budget_bytes);
  if (!s) return PD_ENOMEM;
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
  if (!s->policy.fits_alone(job->io_bytes, job->plan_bytes)) {
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
  if (peak_bytes) *peak_bytes = s->policy.peak();
  if (cache_hits) *cache_hits = s->policy.hits();
  if (cache_misses) *cache_misses = s->policy.misses();
  if (current) *current = s->policy.used();
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
  for (auto &kv : s->policy.cache()) (void)paradiag_plan_destroy(kv.second.handle);
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return PD_OK;
}

// Replay of the admission policy on a scripted sequence of arrivals and
// completions, with `workers` requests running at most at once: the same
// policy object pd_server uses, with no device work.
extern "C" pd_status pd_admission_replay(size_t budget_bytes, int workers,
                                         const pd_admission_event *events, int nevents,
                                         pd_admission_outcome *outcomes, int nreq,
                                         size_t *peak_bytes) {
  if (budget_bytes == 0 || workers < 1 || nevents < 0 || nreq < 0 || (nevents > 0 && !events) ||
      (nreq > 0 && !outcomes)) {
    pd_set_error("pd_admission_replay: invalid arguments");
    return PD_EINVAL;
  }
  using Policy = pdserve::Admission<int, int>;
  Policy policy(budget_bytes);
  struct Req {
    int key = 0;
    size_t io = 0, plan = 0;
    int state = 0;   // 0 unseen, 1 queued, 2 running, 3 finished, 4 rejected
    Policy::Grant grant;
  };
  std::vector<Req> reqs((size_t)nreq);
  std::deque<int> queue;
  int running = 0;
  for (int r = 0; r < nreq; ++r) {
    outcomes[r].admitted_after = -1;
    outcomes[r].cache_hit = 0;
    outcomes[r].evicted = 0;
    outcomes[r].first_victim_key = -1;
    outcomes[r].used_after = 0;
  }
  for (int e = 0; e < nevents; ++e) {
    const pd_admission_event &ev = events[e];
    if (ev.id < 0 || ev.id >= nreq) {
      pd_set_error("pd_admission_replay: request id out of range");
      return PD_EINVAL;
    }
    Req &r = reqs[(size_t)ev.id];
    if (ev.op == 0) {
      if (r.state != 0) {
        pd_set_error("pd_admission_replay: request arrives twice");
        return PD_EINVAL;
      }
      r.key = ev.key;
      r.io = ev.io_bytes;
      r.plan = ev.plan_bytes;
      if (!policy.fits_alone(r.io, r.plan)) {
        r.state = 4;
        outcomes[ev.id].admitted_after = -2;
      } else {
        r.state = 1;
        queue.push_back(ev.id);
      }
    } else if (ev.op == 1) {
      if (r.state != 2) {
        pd_set_error("pd_admission_replay: a request finishes that is not running");
        return PD_EINVAL;
      }
      policy.finish(r.grant, r.key, ev.create_fails == 0, ev.id);
      r.state = 3;
      --running;
    } else {
      pd_set_error("pd_admission_replay: unknown event op");
      return PD_EINVAL;
    }
    // admit from the head of the queue while a worker is free and it fits
    while (running < workers && !queue.empty()) {
      const int id = queue.front();
      Req &h = reqs[(size_t)id];
      std::vector<std::pair<int, int>> evicted;
      h.grant = policy.try_admit(h.key, h.io, h.plan, &evicted);
      if (!h.grant.admitted) break;
      queue.pop_front();
      h.state = 2;
      ++running;
      outcomes[id].admitted_after = e;
      outcomes[id].cache_hit = h.grant.hit ? 1 : 0;
      outcomes[id].evicted = (int)evicted.size();
      outcomes[id].first_victim_key = evicted.empty() ? -1 : evicted.front().first;
      outcomes[id].used_after = policy.used();
    }
  }
  if (peak_bytes) *peak_bytes = policy.peak();
  return PD_OK;
}
