// CPU replay of the persistent batched apply's work order (the host header
// that builds it, compiled without HIP).  Prints one line per check:
//   ok <name>        the check held
//   FAIL <name> ...  it did not
// and, for the planted reversed order, whether the replay found the deadlock.
#include <cstdio>
#include <random>
#include <vector>

#include "persistent_sched.h"

using namespace bfmht;

static std::vector<PSegInfo> random_batch(std::mt19937_64 &rng) {
  std::vector<PSegInfo> segs;
  const int count = 1 + (int)(rng() % 12);
  for (int i = 0; i < count; ++i) {
    const int stages = 2 + (int)(rng() % 11);
    for (int k = 0; k < stages; ++k) {
      // some stages have no items (folded identity levels, empty levels)
      const int64_t pq = (rng() % 5 == 0) ? 0 : 1 + (int64_t)(rng() % 9);
      segs.push_back({i, k, pq});
    }
  }
  return segs;
}

int main() {
  std::mt19937_64 rng(7);
  int fails = 0;
  // 1. every dependency is listed earlier, needs all items of an earlier stage of the same instance
  for (int b = 0; b < 200; ++b) {
    const auto segs = random_batch(rng);
    const PSchedule S = build_schedule(segs);
    for (size_t p = 0; p < S.seg.size(); ++p) {
      const int d = S.dep[p];
      if (d < 0) continue;
      const PSegInfo &a = segs[S.seg[p]], &c = segs[S.seg[d]];
      if (!(d < (int)p && c.inst == a.inst && c.stage < a.stage && S.need[p] == c.per_queue * kQueues)) {
        std::printf("FAIL order batch %d position %zu\n", b, p);
        ++fails;
      }
    }
  }
  std::printf(fails ? "FAIL dependencies\n" : "ok dependencies\n");
  // 2. replays with fewer resident workgroups than items always finish
  int runs = 0, bad = 0;
  for (int b = 0; b < 200; ++b) {
    const auto segs = random_batch(rng);
    const PSchedule S = build_schedule(segs);
    for (int resident = 1; resident <= 3; ++resident)
      for (uint64_t seed = 0; seed < 5; ++seed) {
        int64_t steps = 0;
        ++runs;
        if (!simulate(S, resident, seed * 131 + b, &steps)) ++bad;
      }
  }
  std::printf(bad ? "FAIL replay %d of %d deadlocked\n" : "ok replay %d runs\n", bad ? bad : runs, runs);
  fails += bad;
  // 3. a planted mistake: the same segments listed in reverse stage order make
  //    items wait for items listed after them; the replay must find a deadlock
  int found = 0;
  for (int b = 0; b < 50; ++b) {
    auto segs = random_batch(rng);
    PSchedule S = build_schedule(segs);
    const int n = (int)S.seg.size();
    PSchedule R;
    std::vector<int32_t> newpos(n);
    for (int p = 0; p < n; ++p) newpos[p] = n - 1 - p;
    R.seg.resize(n); R.dep.resize(n); R.need.resize(n); R.item0.resize(n);
    for (int p = 0; p < n; ++p) {
      R.seg[newpos[p]] = S.seg[p];
      R.dep[newpos[p]] = S.dep[p] < 0 ? -1 : newpos[S.dep[p]];
      R.need[newpos[p]] = S.need[p];
    }
    int64_t t = 0;
    for (int p = 0; p < n; ++p) { R.item0[p] = t; t += segs[R.seg[p]].per_queue; }
    R.per_queue_total = t;
    int64_t steps = 0;
    bool any_dep = false;
    for (int p = 0; p < n; ++p) any_dep = any_dep || R.dep[p] >= 0;
    if (any_dep && !simulate(R, 1, b, &steps)) ++found;
  }
  std::printf(found ? "ok reversed order deadlocks %d\n" : "FAIL reversed order never deadlocked\n", found);
  if (!found) ++fails;
  return fails ? 1 : 0;
}
