// serve_policy.h -- the admission rule and the graph-cache eviction rule of the serving
// loop (rfi_server_*, include/rfi.h), free of HIP so that they can be tested on a machine
// without a GPU.
#pragma once

#include <cstddef>
#include <cstdint>
#include <set>

namespace rfi {

// Position in `queue` (FIFO order) of the first request that may be admitted now, or -1.
// A request waits while an earlier request of its plan is still queued or running, or while
// its footprint does not fit in what is left of `budget`; a request that waits also holds
// back the later requests of its plan (per-plan order keeps an array's adaptive state
// updates in integration order), but not those of other plans.  `plan_of(entry)` and
// `bytes_of(entry)` read a queue entry; `running(plan)` tells whether a request of that plan
// is on the device.  Requires inflight_bytes <= budget.
template <class Queue, class PlanOf, class BytesOf, class Running>
std::ptrdiff_t first_admissible(const Queue &queue, PlanOf plan_of, BytesOf bytes_of, Running running,
                                uint64_t inflight_bytes, uint64_t budget) {
  const uint64_t room = budget - inflight_bytes;
  std::set<const void *> held;
  std::ptrdiff_t i = 0;
  for (const auto &entry : queue) {
    const void *plan = plan_of(entry);
    if (held.count(plan) == 0 && !running(plan) && bytes_of(entry) <= room) return i;
    held.insert(plan);
    ++i;
  }
  return -1;
}

// The cached graph to free when the cache is full: the least recently used entry that no
// busy slot is replaying and that is not `keep` (the key about to be captured), or
// cache.end() when every entry is in use.  `cache` maps keys to entries with a `last_use`
// counter; `in_use(key)` tells whether a request on the device replays that key's graph.
// Graphs of destroyed plans are never used again, so they are the first to go.
template <class Cache, class Key, class InUse>
typename Cache::const_iterator graph_to_evict(const Cache &cache, const Key &keep, InUse in_use) {
  auto victim = cache.end();
  for (auto it = cache.begin(); it != cache.end(); ++it) {
    if (!(it->first < keep) && !(keep < it->first)) continue;
    if (in_use(it->first)) continue;
    if (victim == cache.end() || it->second.last_use < victim->second.last_use) victim = it;
  }
  return victim;
}

}  // namespace rfi
