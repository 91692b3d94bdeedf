// Bookkeeping of a profiling window (ssfm_profile_begin .. ssfm_profile_end):
// a pool of event pairs reused across windows, and one record per launch
// that completed, naming the pair of events that brackets it.
//
// Host-only and independent of HIP (the event type is a parameter), so the
// pairing logic is unit-tested on the CPU.  A launch that fails after its
// pair was reserved leaves no record and gives the pair back, so every
// record's events bracket exactly its own launch.
#pragma once

#include <stddef.h>

#include <vector>

namespace ssfm {

template <typename Ev>
class LaunchLog {
 public:
  struct Record {
    int kind;      // kernel family
    double bytes;  // algorithmic HBM bytes of the launch
    size_t pair;   // events 2 pair (before) and 2 pair + 1 (after)
  };

  // Reserve the next event pair, growing the pool with create(Ev*) -> bool.
  // Returns false (and reserves nothing) if an event cannot be created.
  template <typename Create>
  bool reserve(Create&& create, size_t* pair) {
    const size_t need = 2 * (pairs_used_ + 1);
    while (pool_.size() < need) {
      Ev e{};
      if (!create(&e)) return false;
      pool_.push_back(e);
    }
    *pair = pairs_used_++;
    return true;
  }
  // The launch bracketed by `pair` completed.
  void record(size_t pair, int kind, double bytes) { recs_.push_back({kind, bytes, pair}); }
  // The launch of `pair` failed: the pair is free again (it is the last one
  // reserved, since launches are recorded one at a time).
  void release(size_t pair) {
    if (pair + 1 == pairs_used_) --pairs_used_;
  }
  Ev before(const Record& r) const { return pool_[2 * r.pair]; }
  Ev after(const Record& r) const { return pool_[2 * r.pair + 1]; }
  const std::vector<Record>& records() const { return recs_; }
  const std::vector<Ev>& pool() const { return pool_; }
  // A new window: records cleared, the pool kept for reuse.
  void clear() {
    recs_.clear();
    pairs_used_ = 0;
  }

 private:
  std::vector<Ev> pool_;
  size_t pairs_used_ = 0;
  std::vector<Record> recs_;
};

}  // namespace ssfm
