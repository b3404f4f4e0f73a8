// Host-only admission and eviction policy of the serving runtime (no HIP
// calls): the device-memory accounting behind pd_server and the policy replay
// entry point pd_admission_replay.
//
// Accounted bytes = the u0/F/U arrays of every running request + the
// workspace of every plan in the cache (idle or in use).  A request is
// admitted when its need fits the budget: its arrays, plus its plan's bytes
// unless an idle cached plan for the same problem can be reused.  If it does
// not fit, idle cached plans are evicted, least recently used first, until it
// does; if even that is not enough it waits.  Plans in use are never evicted.
#pragma once

#include <cstddef>
#include <map>
#include <utility>
#include <vector>

namespace pdserve {

template <typename Key, typename Handle>
class Admission {
 public:
  struct Entry {
    Handle handle{};
    size_t bytes = 0;
    bool busy = false;
    unsigned long last_used = 0;
  };
  using Cache = std::multimap<Key, Entry>;
  using Iter = typename Cache::iterator;

  // The outcome of an admission attempt.  slot: the reused cache entry
  // (cache().end() when a new plan is to be created).
  struct Grant {
    bool admitted = false;
    bool hit = false;
    Iter slot;
    size_t io = 0, plan_bytes = 0, need = 0;
  };

  explicit Admission(size_t budget) : budget_(budget) {}

  size_t budget() const { return budget_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  long hits() const { return hits_; }
  long misses() const { return misses_; }
  Cache &cache() { return cache_; }

  // A request whose arrays and plan can never fit is rejected up front.
  bool fits_alone(size_t io, size_t plan_bytes) const { return io + plan_bytes <= budget_; }

  // Try to admit a request for `key`.  The handles of evicted plans are
  // appended to *evicted (with their keys) for the caller to free.
  Grant try_admit(const Key &key, size_t io, size_t plan_bytes,
                  std::vector<std::pair<Key, Handle>> *evicted) {
    Grant g;
    g.io = io;
    g.plan_bytes = plan_bytes;
    g.slot = idle_slot(key);
    g.need = io + (g.slot == cache_.end() ? plan_bytes : 0);
    if (used_ + g.need > budget_) {
      if (!make_room(g.need, g.slot, evicted)) {
        g.slot = cache_.end();
        return g;
      }
    }
    g.admitted = true;
    used_ += g.need;
    if (used_ > peak_) peak_ = used_;
    if (g.slot != cache_.end()) {
      g.slot->second.busy = true;
      g.hit = true;
      ++hits_;
    } else {
      ++misses_;
    }
    return g;
  }

  // The admitted request has finished: its arrays are released; a reused
  // plan becomes idle again, a newly created one (created = true) joins the
  // cache with its bytes still accounted, and a failed creation releases
  // its reservation.
  void finish(const Grant &g, const Key &key, bool created, Handle plan) {
    used_ -= g.io;
    if (g.hit) {
      g.slot->second.busy = false;
      g.slot->second.last_used = ++clock_;
    } else if (created) {
      Entry e;
      e.handle = plan;
      e.bytes = g.plan_bytes;
      e.last_used = ++clock_;
      cache_.emplace(key, e);
    } else {
      used_ -= g.plan_bytes;
    }
  }

 private:
  Iter idle_slot(const Key &key) {
    auto range = cache_.equal_range(key);
    for (auto it = range.first; it != range.second; ++it)
      if (!it->second.busy) return it;
    return cache_.end();
  }

  // Evict idle cached plans (least recently used first, never `keep`, the
  // plan the request itself will reuse) until `need` more bytes fit; false
  // if the idle plans do not free enough.
  bool make_room(size_t need, Iter keep, std::vector<std::pair<Key, Handle>> *evicted) {
    size_t idle = 0;
    for (auto it = cache_.begin(); it != cache_.end(); ++it)
      if (!it->second.busy && it != keep) idle += it->second.bytes;
    if (used_ - idle + need > budget_) return false;   // nothing is evicted in vain
    while (used_ + need > budget_) {
      auto victim = cache_.end();
      for (auto it = cache_.begin(); it != cache_.end(); ++it)
        if (!it->second.busy && it != keep &&
            (victim == cache_.end() || it->second.last_used < victim->second.last_used))
          victim = it;
      if (victim == cache_.end()) return false;
      used_ -= victim->second.bytes;
      if (evicted) evicted->emplace_back(victim->first, victim->second.handle);
      cache_.erase(victim);
    }
    return true;
  }

  size_t budget_;
  size_t used_ = 0, peak_ = 0;
  long hits_ = 0, misses_ = 0;
  unsigned long clock_ = 0;
  Cache cache_;
};

}  // namespace pdserve
