// Work order of the persistent batched apply (host side; no HIP).
//
// A persistent batched apply runs every stage of every instance in one launch.
// Its work items (one output tile and column tile of one stage of one
// instance) are handed out through kQueues ticket queues, one per XCD: the
// stage's tile list is already split into kQueues interleaved bins (tile
// 8 s + x belongs to bin x), and queue x holds bin x of every stage.  All
// queues list the segments (instance, stage) in the same order, stage-major:
// stage k of every instance before stage k + 1 of any instance, so an item is
// listed after every item it depends on, in every queue.
//
// A workgroup serving queue x takes its next ticket only after finishing its
// current item, and an item waits only for the items of its instance's
// previous stage (a per-segment count of finished items).  Every item waited
// on is listed earlier; by induction over the stages it is either held by a
// running workgroup whose own wait ends, or not yet taken while its queue
// still has a workgroup that is not blocked (a blocked workgroup holds an item
// listed after it).  So the launch finishes with any number of resident
// workgroups, as long as every queue is served by at least one; nothing
// depends on all workgroups being resident at once.
//
// This header builds that order; the simulation below replays it on the CPU
// with a given number of resident workgroups and a random interleaving.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <random>
#include <vector>

namespace bfmht {

constexpr int kQueues = 8;

// One segment: stage `stage` of instance `inst`, with `per_queue` items in
// each queue (its tile list has 8 per_queue / ny tiles, ny column tiles each).
struct PSegInfo {
  int32_t inst;
  int32_t stage;
  int64_t per_queue;
};

struct PSchedule {
  std::vector<int32_t> seg;     // per position: the segment listed there
  std::vector<int64_t> item0;   // per position: first per-queue ticket of that segment
  std::vector<int32_t> dep;     // per position: position of the segment it waits for, -1 none
  std::vector<int64_t> need;    // per position: finished items (all queues) the wait requires
  int64_t per_queue_total = 0;  // tickets per queue
};

// Stage-major order of the segments with items; each waits for its instance's
// latest earlier stage that has items (stages without items are left out: they
// write nothing).
inline PSchedule build_schedule(const std::vector<PSegInfo> &segs) {
  std::vector<int32_t> idx;
  for (int32_t s = 0; s < (int32_t)segs.size(); ++s)
    if (segs[s].per_queue > 0) idx.push_back(s);
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
    if (segs[a].stage != segs[b].stage) return segs[a].stage < segs[b].stage;
    return segs[a].inst < segs[b].inst;
  });
  PSchedule S;
  std::vector<int32_t> last_pos;   // per instance: position of its latest listed segment
  for (int32_t p = 0; p < (int32_t)idx.size(); ++p) {
    const PSegInfo &g = segs[idx[p]];
    if ((int32_t)last_pos.size() <= g.inst) last_pos.resize(g.inst + 1, -1);
    const int32_t d = last_pos[g.inst];
    S.seg.push_back(idx[p]);
    S.item0.push_back(S.per_queue_total);
    S.dep.push_back(d);
    S.need.push_back(d >= 0 ? segs[S.seg[d]].per_queue * kQueues : 0);
    S.per_queue_total += g.per_queue;
    last_pos[g.inst] = p;
  }
  return S;
}

// Position of the segment that per-queue ticket t belongs to (binary search).
inline int32_t position_of(const PSchedule &S, int64_t t) {
  int32_t lo = 0, hi = (int32_t)S.item0.size() - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (S.item0[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// CPU model of one launch with `resident` workgroups per queue.  At every step
// one workgroup chosen at random acts: an idle one takes its queue's next
// ticket (or retires when the queue is empty), a waiting one starts its item
// once the count it waits for is reached, a working one finishes its item
// (its segment's count goes up).  Returns true when every item finished;
// false on a state where no workgroup can act (a deadlock).  *steps counts
// the actions taken.
inline bool simulate(const PSchedule &S, int resident, uint64_t seed, int64_t *steps) {
  struct WG { int q; int state; int64_t ticket; int32_t pos; };   // state 0 idle, 1 waiting, 2 working, 3 retired
  std::vector<WG> wg;
  for (int q = 0; q < kQueues; ++q)
    for (int r = 0; r < resident; ++r) wg.push_back({q, 0, -1, -1});
  std::vector<int64_t> head(kQueues, 0), done(S.seg.size(), 0);
  std::mt19937_64 rng(seed);
  int64_t n = 0, finished = 0;
  const int64_t total = S.per_queue_total * kQueues;
  while (finished < total) {
    std::vector<int> can;
    for (int w = 0; w < (int)wg.size(); ++w) {
      const WG &g = wg[w];
      if (g.state == 0 || g.state == 2) can.push_back(w);
      else if (g.state == 1 && (S.dep[g.pos] < 0 || done[S.dep[g.pos]] >= S.need[g.pos])) can.push_back(w);
    }
    if (can.empty()) {
      if (steps) *steps = n;
      return false;
    }
    WG &g = wg[can[rng() % can.size()]];
    if (g.state == 0) {
      if (head[g.q] >= S.per_queue_total) {
        g.state = 3;
      } else {
        g.ticket = head[g.q]++;
        g.pos = position_of(S, g.ticket);
        g.state = 1;
      }
    } else if (g.state == 1) {
      g.state = 2;
    } else {
      ++done[g.pos];
      ++finished;
      g.state = 0;
    }
    ++n;
  }
  if (steps) *steps = n;
  return true;
}

}  // namespace bfmht
