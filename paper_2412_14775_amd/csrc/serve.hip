// serve.hip -- the persistent request loop of librfi (rfi_server_*, include/rfi.h).
//
// One scheduler thread owns the queues.  Requests wait in a time-ordered set
// until their arrival time, then in a FIFO queue until a slot (a HIP stream)
// is free and the summed footprint of admitted requests leaves room for them;
// requests of one plan stay in order.  An admitted request replays a captured
// hipGraph of its screen step on its slot's stream, followed by a host
// callback that timestamps completion and frees the slot.  The callback takes
// the server mutex only briefly and never calls into HIP.
//
// Tracing: each admission is a roctx range ("rfi_server admit tag=... slot=..." around the
// graph launch or capture and the callback's enqueue), each capture and each completion a
// roctx mark, so a rocprofv3 --marker-trace run lines requests up with their kernels.  With
// no profiler attached the calls do nothing.

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <chrono>
#include <cinttypes>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <atomic>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/rfi.h"
#include "internal.h"
#include "plan.h"
#include "serve_policy.h"

namespace {

using Clock = std::chrono::steady_clock;

// A cached graph holds the plan's kernel arguments, so it is keyed by the plan's
// uid (never reused) rather than its address (reused once a plan is destroyed).
struct GraphKey {
  uint64_t plan;
  const void *vis, *avg, *weight, *flags, *stats;
  bool operator<(const GraphKey &o) const {
    return std::tie(plan, vis, avg, weight, flags, stats) < std::tie(o.plan, o.vis, o.avg, o.weight, o.flags, o.stats);
  }
};

struct CachedGraph {
  hipGraph_t graph;
  hipGraphExec_t exec;
  uint64_t last_use;  // scheduler's use counter at the last replay
};

constexpr int32_t kDefaultMaxGraphs = 256;

GraphKey key_of(const rfi_request &r) {
  return GraphKey{rfi::plan_uid(r.plan), r.vis, r.avg, r.weight, r.flags, r.stats};
}

struct Pending {
  rfi_request req;
  uint64_t bytes;
  uint64_t seq;
};

struct SlotCtx {
  rfi_server *srv;
  int slot;
};

int set_error(int code, const char *msg) { return rfi::set_error(code, "%s", msg); }

}  // namespace

struct rfi_server {
  rfi_server_config cfg{};
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_sched;
  std::condition_variable cv_done;
  std::multimap<double, Pending> future;   // not yet arrived
  std::deque<Pending> queue;               // arrived, waiting for admission
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  std::vector<const rfi_plan *> slot_plan;
  std::vector<uint64_t> slot_bytes;
  std::vector<rfi_completion> slot_rec;
  std::vector<GraphKey> slot_key;          // graph key of each busy slot's request
  std::vector<SlotCtx> ctx;
  std::deque<rfi_completion> done;
  // Captured graphs, touched by the scheduler thread only (and by rfi_server_destroy after
  // it has joined): at most max_graphs of them, the least recently used not on the device
  // freed first, so a long run with fresh buffers or short-lived plans stays bounded.
  std::map<GraphKey, CachedGraph> graphs;
  int32_t max_graphs = kDefaultMaxGraphs;
  uint64_t use_clock = 0;
  std::atomic<int> n_cached{0};
  uint64_t inflight_bytes = 0;
  int inflight = 0;
  uint64_t outstanding = 0;
  uint64_t seq = 0;
  uint64_t events = 0;  // bumped by every submit and completion: the scheduler re-plans on change
  rfi_server_stats stats{};
  std::atomic<int> n_graphs{0};
  bool stop = false;
  std::thread thread;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void run();
  int launch(int slot, const rfi_request &r);
  static void on_done(void *p);
};

// Host callback after a request's graph: runs on a runtime thread, no HIP calls.
void rfi_server::on_done(void *p) {
  SlotCtx *c = static_cast<SlotCtx *>(p);
  rfi_server *s = c->srv;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    rfi_completion rec = s->slot_rec[c->slot];
    char msg[80];
    std::snprintf(msg, sizeof msg, "rfi_server done tag=%" PRIu64 " slot=%d", rec.tag, c->slot);
    roctxMarkA(msg);
    rec.done = s->now();
    s->done.push_back(rec);
    s->slot_busy[c->slot] = false;
    s->slot_plan[c->slot] = nullptr;
    s->inflight_bytes -= s->slot_bytes[c->slot];
    s->inflight -= 1;
    s->outstanding -= 1;
    s->stats.completed += 1;
    s->events += 1;
  }
  s->cv_sched.notify_one();
  s->cv_done.notify_all();
}

int rfi_server::launch(int slot, const rfi_request &r) {
  hipStream_t st = streams[slot];
  if (!cfg.use_graphs) return rfi_screen(r.plan, r.vis, r.avg, r.weight, r.flags, r.stats, st);
  const GraphKey key = key_of(r);
  auto it = graphs.find(key);
  if (it == graphs.end()) {
    if ((int64_t)graphs.size() >= max_graphs) {
      // pick the victim under the mutex (slot_busy / slot_key), free it without: a slot that
      // is not busy has run its completion callback, which follows its graph on the stream
      auto victim = graphs.cend();
      {
        std::lock_guard<std::mutex> lk(mu);
        auto in_use = [this](const GraphKey &k) {
          for (int s = 0; s < cfg.n_slots; ++s)
            if (slot_busy[s] && !(slot_key[s] < k) && !(k < slot_key[s])) return true;
          return false;
        };
        victim = rfi::graph_to_evict(graphs, key, in_use);
      }
      if (victim != graphs.cend()) {
        (void)hipGraphExecDestroy(victim->second.exec);
        (void)hipGraphDestroy(victim->second.graph);
        graphs.erase(victim);
      }
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    roctxMarkA("rfi_server capture graph");
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(RFI_ERR_DEVICE, "hipStreamBeginCapture failed");
    const int rc = rfi_screen(r.plan, r.vis, r.avg, r.weight, r.flags, r.stats, st);
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (rc != RFI_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc != RFI_OK ? rc : set_error(RFI_ERR_DEVICE, "hipStreamEndCapture failed");
    }
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return set_error(RFI_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    it = graphs.emplace(key, CachedGraph{g, ge, 0}).first;
    n_graphs.fetch_add(1);
  }
  it->second.last_use = ++use_clock;
  n_cached.store((int)graphs.size());
  if (hipGraphLaunch(it->second.exec, st) != hipSuccess) return set_error(RFI_ERR_DEVICE, "hipGraphLaunch failed");
  return RFI_OK;
}

void rfi_server::run() {
  (void)hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    const uint64_t seen = events;
    const double t = now();
    while (!future.empty() && future.begin()->first <= t) {
      queue.push_back(future.begin()->second);
      future.erase(future.begin());
    }
    // admission: FIFO, skipping requests that cannot go yet; a plan stays in order
    // (rfi::first_admissible); one request per free slot
    auto plan_of = [](const Pending &q) { return static_cast<const void *>(q.req.plan); };
    auto bytes_of = [](const Pending &q) { return q.bytes; };
    auto running = [this](const void *plan) {
      for (int s = 0; s < cfg.n_slots; ++s)
        if (slot_busy[s] && slot_plan[s] == plan) return true;
      return false;
    };
    for (;;) {
      int slot = -1;
      for (int s = 0; s < cfg.n_slots; ++s)
        if (!slot_busy[s]) {
          slot = s;
          break;
        }
      if (slot < 0) break;
      const std::ptrdiff_t k = rfi::first_admissible(queue, plan_of, bytes_of, running, inflight_bytes, cfg.hbm_budget);
      if (k < 0) break;
      const Pending p = queue[k];
      const rfi_plan *plan = p.req.plan;
      queue.erase(queue.begin() + k);  // only this thread touches `queue`
      slot_busy[slot] = true;
      slot_plan[slot] = plan;
      slot_key[slot] = key_of(p.req);
      slot_bytes[slot] = p.bytes;
      inflight_bytes += p.bytes;
      inflight += 1;
      if (inflight_bytes > stats.peak_inflight_bytes) stats.peak_inflight_bytes = inflight_bytes;
      if (inflight > stats.peak_inflight) stats.peak_inflight = inflight;
      rfi_completion &rec = slot_rec[slot];
      rec.tag = p.req.tag;
      rec.slot = slot;
      rec.arrival = p.req.arrival;
      rec.admitted = now();
      rec.done = 0.0;
      rec.status = RFI_OK;
      // HIP calls run without the mutex: the completion callback takes it
      lk.unlock();
      char msg[80];
      std::snprintf(msg, sizeof msg, "rfi_server admit tag=%" PRIu64 " slot=%d", p.req.tag, slot);
      roctxRangePushA(msg);
      int rc = launch(slot, p.req);
      if (rc == RFI_OK && hipLaunchHostFunc(streams[slot], &rfi_server::on_done, &ctx[slot]) != hipSuccess)
        rc = set_error(RFI_ERR_DEVICE, "hipLaunchHostFunc failed");
      roctxRangePop();
      if (rc != RFI_OK) (void)hipStreamSynchronize(streams[slot]);
      lk.lock();
      if (rc != RFI_OK) {  // no callback was enqueued: complete the request here
        rfi_completion r = slot_rec[slot];
        r.status = rc;
        r.done = now();
        done.push_back(r);
        slot_busy[slot] = false;
        slot_plan[slot] = nullptr;
        inflight_bytes -= p.bytes;
        inflight -= 1;
        outstanding -= 1;
        stats.completed += 1;
        stats.failed += 1;
        cv_done.notify_all();
      }
    }
    if (stop && outstanding == 0) break;
    // sleep until something changed since this pass began, or the next arrival is due
    auto changed = [this, seen] { return events != seen || (stop && outstanding == 0); };
    if (!future.empty()) {
      const auto wake = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(future.begin()->first));
      cv_sched.wait_until(lk, wake, changed);
    } else {
      cv_sched.wait(lk, changed);
    }
  }
}

extern "C" {

int rfi_server_create(const rfi_server_config *cfg, rfi_server **out) {
  if (out == nullptr) return set_error(RFI_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (cfg == nullptr) return set_error(RFI_ERR_INVALID_ARGUMENT, "cfg is NULL");
  if (cfg->n_slots < 1 || cfg->n_slots > 64) return set_error(RFI_ERR_INVALID_ARGUMENT, "n_slots must be in 1..64");
  if (cfg->hbm_budget == 0) return set_error(RFI_ERR_INVALID_ARGUMENT, "hbm_budget must be > 0");
  if (cfg->device < 0) return set_error(RFI_ERR_INVALID_ARGUMENT, "device must be >= 0");
  if (cfg->max_graphs < 0) return set_error(RFI_ERR_INVALID_ARGUMENT, "max_graphs must be >= 0 (0: the default)");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || cfg->device >= count)
    return set_error(RFI_ERR_DEVICE, "device not available");
  rfi_server *s = new (std::nothrow) rfi_server();
  if (s == nullptr) return set_error(RFI_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->cfg = *cfg;
  s->max_graphs = cfg->max_graphs > 0 ? cfg->max_graphs : kDefaultMaxGraphs;
  s->t0 = Clock::now();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(cfg->device);
  const int n = cfg->n_slots;
  s->streams.assign(n, nullptr);
  s->slot_busy.assign(n, false);
  s->slot_plan.assign(n, nullptr);
  s->slot_bytes.assign(n, 0);
  s->slot_rec.assign(n, rfi_completion{});
  s->slot_key.assign(n, GraphKey{});
  s->ctx.resize(n);
  for (int i = 0; i < n; ++i) {
    s->ctx[i] = SlotCtx{s, i};
    if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipStreamDestroy(s->streams[j]);
      (void)hipSetDevice(prev);
      delete s;
      return set_error(RFI_ERR_DEVICE, "hipStreamCreateWithFlags failed");
    }
  }
  (void)hipSetDevice(prev);
  s->thread = std::thread([s] { s->run(); });
  *out = s;
  return RFI_OK;
}

double rfi_server_now(const rfi_server *srv) { return srv ? srv->now() : 0.0; }

int rfi_server_submit(rfi_server *srv, const rfi_request *req) {
  if (srv == nullptr || req == nullptr) return set_error(RFI_ERR_INVALID_ARGUMENT, "server and request must not be NULL");
  if (req->plan == nullptr || req->vis == nullptr || req->avg == nullptr || req->weight == nullptr)
    return set_error(RFI_ERR_INVALID_ARGUMENT, "plan, vis, avg and weight must not be NULL");
  if (reinterpret_cast<uintptr_t>(req->vis) % 16 || reinterpret_cast<uintptr_t>(req->avg) % 16)
    return set_error(RFI_ERR_INVALID_ARGUMENT, "vis and avg must be 16-byte aligned");
  size_t bytes = 0;
  if (rfi_plan_footprint(req->plan, &bytes) != RFI_OK) return set_error(RFI_ERR_INVALID_ARGUMENT, "bad plan");
  if (req->stats != nullptr) bytes += rfi::plan_stats_bytes(req->plan);  // optional output
  if (bytes > srv->cfg.hbm_budget)
    return set_error(RFI_ERR_INVALID_ARGUMENT, "request footprint exceeds the server's HBM budget");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return set_error(RFI_ERR_INVALID_ARGUMENT, "server is stopping");
    Pending p{*req, (uint64_t)bytes, srv->seq++};
    srv->future.emplace(req->arrival, p);
    srv->outstanding += 1;
    srv->stats.submitted += 1;
    srv->events += 1;
  }
  srv->cv_sched.notify_one();
  return RFI_OK;
}

int rfi_server_poll(rfi_server *srv, rfi_completion *out, int32_t max, int32_t *n_out, double timeout_s) {
  if (srv == nullptr || n_out == nullptr || (out == nullptr && max > 0))
    return set_error(RFI_ERR_INVALID_ARGUMENT, "server, out and n_out must not be NULL");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (srv->done.empty() && timeout_s > 0)
    srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [srv] { return !srv->done.empty(); });
  int32_t n = 0;
  while (n < max && !srv->done.empty()) {
    out[n++] = srv->done.front();
    srv->done.pop_front();
  }
  *n_out = n;
  return RFI_OK;
}

int rfi_server_drain(rfi_server *srv, double timeout_s) {
  if (srv == nullptr) return set_error(RFI_ERR_INVALID_ARGUMENT, "server is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  const bool ok = srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [srv] { return srv->outstanding == 0; });
  return ok ? RFI_OK : set_error(RFI_ERR_DEVICE, "drain timed out");
}

int rfi_server_get_stats(const rfi_server *srv, rfi_server_stats *out) {
  if (srv == nullptr || out == nullptr) return set_error(RFI_ERR_INVALID_ARGUMENT, "server and out must not be NULL");
  std::lock_guard<std::mutex> lk(const_cast<rfi_server *>(srv)->mu);
  *out = srv->stats;
  out->graphs = srv->n_graphs.load();
  out->graphs_cached = srv->n_cached.load();
  return RFI_OK;
}

int rfi_server_destroy(rfi_server *srv) {
  if (srv == nullptr) return RFI_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->events += 1;
  }
  srv->cv_sched.notify_one();
  if (srv->thread.joinable()) srv->thread.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(srv->cfg.device);
  for (hipStream_t st : srv->streams) (void)hipStreamSynchronize(st);
  for (auto &kv : srv->graphs) {
    (void)hipGraphExecDestroy(kv.second.exec);
    (void)hipGraphDestroy(kv.second.graph);
  }
  for (hipStream_t st : srv->streams) (void)hipStreamDestroy(st);
  (void)hipSetDevice(prev);
  delete srv;
  return RFI_OK;
}

}  // extern "C"
