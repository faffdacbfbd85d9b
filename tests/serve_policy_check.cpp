// The serving loop's admission rule (csrc/serve_policy.h) on fixed cases and in a simulated
// scheduler, without a GPU.  Prints "ALL OK" when every expectation holds.
#include <cstdint>
#include <cstdio>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "serve_policy.h"

static int failures = 0;
#define EXPECT(cond)                                                \
  do {                                                              \
    if (!(cond)) {                                                  \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                   \
    }                                                               \
  } while (0)

struct Req {
  int plan;
  uint64_t bytes;
  int seq;
};

static const int kPlans[8] = {0, 1, 2, 3, 4, 5, 6, 7};  // stable addresses stand for plans

static std::ptrdiff_t pick(const std::deque<Req> &q, const std::vector<int> &running_plans, uint64_t inflight,
                           uint64_t budget) {
  return rfi::first_admissible(
      q, [](const Req &r) { return static_cast<const void *>(&kPlans[r.plan]); },
      [](const Req &r) { return r.bytes; },
      [&](const void *plan) {
        for (int p : running_plans)
          if (plan == &kPlans[p]) return true;
        return false;
      },
      inflight, budget);
}

static void fixed_cases() {
  const uint64_t B = 100;
  EXPECT(pick({}, {}, 0, B) == -1);                                       // nothing queued
  EXPECT(pick({{0, 10, 0}, {1, 10, 1}}, {}, 0, B) == 0);                  // FIFO
  EXPECT(pick({{0, 10, 0}, {0, 10, 1}}, {0}, 0, B) == -1);                // plan running: both wait
  EXPECT(pick({{0, 10, 0}, {1, 10, 1}}, {0}, 0, B) == 1);                 // another plan may go
  EXPECT(pick({{0, 90, 0}, {1, 10, 1}}, {}, 20, B) == 1);                 // too big now: others pass it
  EXPECT(pick({{0, 90, 0}, {0, 10, 1}}, {}, 20, B) == -1);                // ... but not its own plan
  EXPECT(pick({{0, 90, 0}, {0, 10, 1}, {2, 10, 2}}, {}, 20, B) == 2);
  EXPECT(pick({{0, 80, 0}}, {}, 20, B) == 0);                             // exact fit
  EXPECT(pick({{0, 81, 0}}, {}, 20, B) == -1);
  EXPECT(pick({{0, 100, 0}}, {}, 0, B) == 0);                             // the whole budget
  const uint64_t huge = ~uint64_t(0);
  EXPECT(pick({{0, huge - 5, 0}}, {}, 10, huge) == -1);                   // no overflow in the sum
  EXPECT(pick({{0, huge - 10, 0}}, {}, 10, huge) == 0);
}

// A scheduler driven by the rule: random plans, sizes and durations, a few slots, a budget.
// Checks that admissions keep each plan's order, never exceed the budget, never leave a slot
// idle while something admissible waits, and that every request is served.
static void simulation(unsigned seed) {
  std::mt19937 rng(seed);
  const int n_slots = 1 + (int)(rng() % 4), n_req = 400;
  const uint64_t budget = 100;
  std::deque<Req> queue;
  for (int i = 0; i < n_req; ++i) queue.push_back({(int)(rng() % 6), 1 + rng() % budget, i});
  struct Slot {
    bool busy = false;
    int plan = -1;
    uint64_t bytes = 0;
    int left = 0;
  };
  std::vector<Slot> slots(n_slots);
  std::map<int, int> last_seq;  // per plan: sequence number of the last admitted request
  uint64_t inflight = 0;
  int served = 0, ticks = 0;
  while (served < n_req && ticks < 100000) {
    ++ticks;
    for (auto &s : slots)  // completions
      if (s.busy && --s.left == 0) {
        s.busy = false;
        inflight -= s.bytes;
        ++served;
      }
    for (;;) {  // admissions, as the server does them
      int free_slot = -1;
      for (int i = 0; i < n_slots; ++i)
        if (!slots[i].busy) {
          free_slot = i;
          break;
        }
      if (free_slot < 0) break;
      std::vector<int> running;
      for (auto &s : slots)
        if (s.busy) running.push_back(s.plan);
      const std::ptrdiff_t k = pick(queue, running, inflight, budget);
      if (k < 0) {
        // nothing admissible: then every queued request is held by its plan or the budget
        for (size_t i = 0; i < queue.size(); ++i) {
          bool plan_first = true, plan_running = false;
          for (size_t j = 0; j < i; ++j) plan_first &= queue[j].plan != queue[i].plan;
          for (int p : running) plan_running |= p == queue[i].plan;
          EXPECT(!plan_first || plan_running || queue[i].bytes > budget - inflight);
        }
        break;
      }
      const Req r = queue[k];
      queue.erase(queue.begin() + k);
      auto it = last_seq.find(r.plan);
      EXPECT(it == last_seq.end() || it->second < r.seq);  // per-plan order
      last_seq[r.plan] = r.seq;
      inflight += r.bytes;
      EXPECT(inflight <= budget);
      slots[free_slot] = Slot{true, r.plan, r.bytes, 1 + (int)(rng() % 5)};
    }
  }
  EXPECT(served == n_req);
  EXPECT(queue.empty());
}

// The graph-cache eviction rule: least recently used, never a graph on the device, never the
// key about to be captured; none when all are in use.
struct Entry {
  uint64_t last_use;
};

static void eviction_cases() {
  std::map<int, Entry> cache{{1, {5}}, {2, {3}}, {3, {9}}, {4, {1}}};
  auto none = [](int) { return false; };
  EXPECT(rfi::graph_to_evict(cache, 99, none)->first == 4);            // least recently used
  EXPECT(rfi::graph_to_evict(cache, 4, none)->first == 2);             // not the key being captured
  auto busy4 = [](int k) { return k == 4; };
  EXPECT(rfi::graph_to_evict(cache, 99, busy4)->first == 2);           // not one on the device
  auto busy24 = [](int k) { return k == 2 || k == 4; };
  EXPECT(rfi::graph_to_evict(cache, 1, busy24)->first == 3);
  auto all = [](int) { return true; };
  EXPECT(rfi::graph_to_evict(cache, 99, all) == cache.end());          // everything in use
  std::map<int, Entry> empty;
  EXPECT(rfi::graph_to_evict(empty, 1, none) == empty.end());
  // a cache driven like the server's: capacity 3, random uses, some keys "on the device";
  // the cache never holds an in-use key's eviction and stays at capacity
  std::mt19937 rng(7);
  std::map<int, Entry> c;
  uint64_t clock = 0;
  for (int step = 0; step < 2000; ++step) {
    const int key = (int)(rng() % 8);
    const int on_device = (int)(rng() % 8);
    auto in_use = [&](int k) { return k == on_device; };
    if (c.find(key) == c.end()) {
      if (c.size() >= 3) {
        auto v = rfi::graph_to_evict(c, key, in_use);
        EXPECT(v != c.end());
        if (v != c.end()) {
          EXPECT(v->first != key && v->first != on_device);
          for (auto &kv : c)  // nothing older that could have gone
            EXPECT(kv.first == key || kv.first == on_device || kv.second.last_use >= v->second.last_use);
          c.erase(v);
        }
      }
      c[key] = Entry{0};
    }
    c[key].last_use = ++clock;
    EXPECT(c.size() <= 3);
  }
}

int main() {
  fixed_cases();
  eviction_cases();
  for (unsigned seed = 1; seed <= 50; ++seed) simulation(seed);
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("ALL OK\n");
  return 0;
}
