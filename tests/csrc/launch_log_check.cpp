// CPU check of the profiling window's launch bookkeeping (launch_log.hpp):
// event pairs are reserved per launch, a failed launch leaves no record and
// frees its pair, and every record's events are the pair reserved for it.
// Events are stand-in integers; prints "ok" and exits 0 on success.
#include <stdio.h>
#include <stdlib.h>

#include "launch_log.hpp"

#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      return 1;                                                   \
    }                                                             \
  } while (0)

int main() {
  ssfm::LaunchLog<int> log;
  int next = 100;  // event "handles" handed out by the stand-in creator
  int fail_after = -1;
  auto create = [&](int* e) {
    if (fail_after == 0) return false;
    if (fail_after > 0) --fail_after;
    *e = next++;
    return true;
  };
  // launches 0, 1 succeed; 2 fails after its pair was reserved; 3 succeeds
  for (int i = 0; i < 4; ++i) {
    size_t pair = 0;
    CHECK(log.reserve(create, &pair));
    if (i == 2) {
      log.release(pair);
      continue;
    }
    log.record(pair, i, 10.0 * i);
  }
  CHECK(log.records().size() == 3);
  // the failed launch's pair was reused by launch 3: pairs 0, 1, 2
  const int kinds[3] = {0, 1, 3};
  for (size_t k = 0; k < 3; ++k) {
    const auto& r = log.records()[k];
    CHECK(r.kind == kinds[k]);
    CHECK(r.pair == k);
    CHECK(log.before(r) == 100 + 2 * (int)k);
    CHECK(log.after(r) == 101 + 2 * (int)k);
  }
  CHECK(log.pool().size() == 6);
  // a new window reuses the pool without creating events
  log.clear();
  CHECK(log.records().empty());
  for (int i = 0; i < 3; ++i) {
    size_t pair = 0;
    CHECK(log.reserve(create, &pair));
    log.record(pair, 7, 1.0);
  }
  CHECK(log.pool().size() == 6);
  CHECK(next == 106);
  // growing past the pool: creation failure reserves nothing
  fail_after = 1;  // one more event can be created, the second fails
  size_t pair = 99;
  CHECK(!log.reserve(create, &pair));
  CHECK(pair == 99);
  CHECK(log.records().size() == 3);
  // the next reservation after a failure still yields the next pair
  fail_after = -1;
  CHECK(log.reserve(create, &pair));
  CHECK(pair == 3);
  log.record(pair, 2, 5.0);
  const auto& last = log.records().back();
  CHECK(log.before(last) == log.pool()[6] && log.after(last) == log.pool()[7]);
  puts("ok");
  return 0;
}
