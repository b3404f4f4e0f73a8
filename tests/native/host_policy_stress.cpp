// Stress driver for the host-only C++ of libparadiag, built with the address
// and undefined-behaviour sanitizers by tests/test_host_sanitized_cpu.py:
// random scripts through the serving admission policy (with its accounting
// invariants checked after every step) and random problems through the plan
// validation.  Exits non-zero on the first violated invariant.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2304_12597_amd/csrc/pd_admission.h"
#include "../../paper_2304_12597_amd/csrc/pd_validate.h"

#define CHECK(c)                                                         \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "invariant failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                      \
    }                                                                    \
  } while (0)

static void stress_admission(unsigned seed) {
  std::mt19937 rng(seed);
  const size_t budget = 1000;
  pdserve::Admission<int, int> pol(budget);
  struct Run { int key; size_t io; pdserve::Admission<int, int>::Grant g; };
  std::vector<Run> running;
  size_t io_running = 0;
  for (int step = 0; step < 4000; ++step) {
    if (running.empty() || rng() % 3 != 0) {
      const int key = (int)(rng() % 12);
      const size_t io = 1 + rng() % 300, plan = 1 + rng() % 400;
      if (!pol.fits_alone(io, plan)) continue;
      std::vector<std::pair<int, int>> ev;
      auto g = pol.try_admit(key, io, plan, &ev);
      if (g.admitted) {
        running.push_back({key, io, g});
        io_running += io;
      } else {
        CHECK(ev.empty());
      }
    } else {
      const size_t idx = rng() % running.size();
      Run r = running[idx];
      running.erase(running.begin() + (long)idx);
      io_running -= r.io;
      pol.finish(r.g, r.key, rng() % 10 != 0, step);
    }
    size_t cached = 0, busy = 0;
    for (auto &kv : pol.cache()) {
      cached += kv.second.bytes;
      busy += kv.second.busy ? 1 : 0;
    }
    size_t hits_running = 0;
    for (auto &r : running) hits_running += r.g.hit ? 1 : 0;
    size_t plans_reserved = 0;
    for (auto &r : running) plans_reserved += r.g.hit ? 0 : r.g.plan_bytes;
    CHECK(busy == hits_running);
    CHECK(pol.used() == io_running + cached + plans_reserved);
    CHECK(pol.used() <= budget);
    CHECK(pol.peak() <= budget);
  }
}

static void stress_validation(unsigned seed) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> u(-2.0, 2.0);
  for (int it = 0; it < 3000; ++it) {
    const int n = 1 + (int)(rng() % 40);
    std::vector<double> kl(n), kd(n), ku(n), ml(n), md(n), mu(n);
    for (int i = 0; i < n; ++i) {
      kl[i] = u(rng); kd[i] = u(rng); ku[i] = u(rng);
      ml[i] = u(rng); md[i] = 4.0 + u(rng); mu[i] = u(rng);
    }
    if (rng() % 5 == 0) kd[rng() % n] = 0.0 / 0.0;
    pd_tridiag K{kl.data(), kd.data(), ku.data()}, M{ml.data(), md.data(), mu.data()};
    pd_options opt{};
    opt.dims = 1 + (int)(rng() % 3);
    opt.precision = (int)(rng() % 4);
    opt.alpha = (rng() % 2) ? 1.0 : u(rng);
    opt.maxit = (int)(rng() % 70);
    opt.max_sweeps = (int)(rng() % 70);
    opt.krylov = (int)(rng() % 3);
    opt.fom_q = (int)(rng() % 3);
    opt.bdf_order = (int)(rng() % 8);
    opt.shifted_solver = (int)(rng() % 3);
    const int ell = 1 << (rng() % 14);
    std::string msg;
    const pd_status st = pdcheck::check_plan_args(n, ell, 0.01 + u(rng), (rng() % 2) ? &M : nullptr,
                                                  &K, opt, &msg);
    CHECK(st == PD_OK || !msg.empty());
  }
}

int main() {
  for (unsigned s = 0; s < 8; ++s) {
    stress_admission(s);
    stress_validation(s);
  }
  std::printf("host policy stress: ok\n");
  return 0;
}
