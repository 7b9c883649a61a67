// Serving loop of libsta: resident designs, an admission queue against a device-memory
// budget, and continuous batching of requests over per-slot HIP streams.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "sta_internal.h"

using namespace sta;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Pinned host buffers reused by exact size (designs repeat, so sizes do too).
class PinnedPool {
 public:
  void* take(size_t bytes) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = free_.find(bytes);
      if (it != free_.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        return p;
      }
    }
    void* p = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    const hipError_t e = hipHostMalloc(&p, std::max<size_t>(bytes, 1), hipHostMallocDefault);
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::lock_guard<std::mutex> lk(mu_);
    ++allocs_;
    alloc_ms_ += ms;
    return e == hipSuccess ? p : nullptr;
  }
  void counts(int64_t* n, double* ms) {
    std::lock_guard<std::mutex> lk(mu_);
    *n = allocs_;
    *ms = alloc_ms_;
  }
  void give(void* p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_[bytes].push_back(p);
  }
  ~PinnedPool() {
    for (auto& kv : free_)
      for (void* p : kv.second) (void)hipHostFree(p);
  }

 private:
  std::mutex mu_;
  std::map<size_t, std::vector<void*>> free_;
  int64_t allocs_ = 0;     // hipHostMalloc calls and their host time
  double alloc_ms_ = 0.0;
};

struct Design {
  sta_graph* g = nullptr;
  int P = 0;
  float* x = nullptr;   // resident coordinates (device, original order)
  float* y = nullptr;
  size_t state_bytes = 0, work_bytes = 0;   // of one snapshot
  bool can_merge = false;                   // snapshot-outer layout with lane-group schedules
};

enum TicketState { kQueued, kRunning, kDone, kFailed };

struct Ticket {
  int design = 0, kind = 0, P = 0;
  float gamma = 10.f;
  TicketState st = kQueued;
  sta_status err = STA_OK;
  std::string msg;
  float* hx = nullptr;   // pinned staging of new coordinates, or NULL
  float* hy = nullptr;
  double* hsc = nullptr; // pinned results
  float* hdx = nullptr;
  float* hdy = nullptr;
  size_t need = 0;       // device bytes of its buffers
  int slot = -1;
  Clock::time_point t_submit, t_admit, t_done;
};

// A slot runs one sweep at a time on its own stream, in a device buffer it keeps between
// sweeps, with the launch sequence of each (design, kind, coordinates, gamma, snapshots)
// captured once into a hipGraph over that buffer and replayed afterwards.  A sweep serves
// one request, or several of one design, kind and gamma as its snapshots.
using GraphKey = std::tuple<int, int, int, uint32_t, int>;   // (design, kind, new x/y, gamma bits, S)
constexpr size_t kMaxSlotGraphs = 128;  // captured sequences kept per slot; the oldest goes first

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  std::vector<uint64_t> batch;  // tickets of the sweep on the device, snapshot order
  bool busy = false;
  void* buf = nullptr;          // from the server's pool
  size_t cap = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::deque<GraphKey> graph_order;   // capture order, for eviction
};

// What issuing a sweep needs, copied out of the tickets and the design table so that the
// scheduler can capture and enqueue without holding the server's lock.
struct Member {                 // one request (snapshot) of the sweep
  const float *hx, *hy;         // pinned new coordinates, or NULL: the design's
  float *hdx, *hdy;
  double* hsc;
};
struct Issue {
  int design, kind;
  float gamma;
  int S;                        // snapshots: 1 runs the request's own graph of one snapshot
  bool new_xy;                  // the sweep reads coordinates from its buffer (always when S > 1)
  std::vector<Member> m;
};

// Where a request's buffers sit inside its slot's buffer.
struct Carve {
  void* state;
  double* sc;
  void* ws;
  float *dx, *dy, *x, *y;
};

}  // namespace

struct sta_server {
  sta_server_config cfg{};
  int device = -1;
  hipMemPool_t pool = nullptr;
  hipStream_t setup_stream = nullptr;
  std::vector<Slot> slots;
  std::vector<Design> designs;
  size_t resident = 0;        // bytes of designs (graph copies and coordinates)
  hipStream_t cap_stream = nullptr;   // captures the slots' launch sequences
  std::mutex mu;
  std::condition_variable wake;       // scheduler: new work or stop
  std::condition_variable finished;   // waiters: a ticket finished
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  PinnedPool pinned;
  sta_server_stats stats{};

  // Device bytes of a sweep of S snapshots (every per-call buffer holds S copies back to back).
  size_t request_bytes(const Design& d, int kind, bool new_xy, int S = 1) const {
    const size_t n = (size_t)S;
    size_t b = align256(n * d.state_bytes) + align256(n * 4 * sizeof(double));
    if (kind == STA_REQ_FWD_BWD) b += align256(n * d.work_bytes) + 2 * align256(n * sizeof(float) * (size_t)d.P);
    if (new_xy || S > 1) b += 2 * align256(n * sizeof(float) * (size_t)d.P);
    return b;
  }

  static Carve carve(void* base, const Design& d, int kind, bool new_xy, int S) {
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) {
      char* r = p;
      p += align256(bytes);
      return r;
    };
    const size_t n = (size_t)S, fb = sizeof(float) * (size_t)d.P;
    Carve c{};
    c.state = take(n * d.state_bytes);
    c.sc = reinterpret_cast<double*>(take(n * 4 * sizeof(double)));
    if (kind == STA_REQ_FWD_BWD) {
      c.ws = take(n * d.work_bytes);
      c.dx = reinterpret_cast<float*>(take(n * fb));
      c.dy = reinterpret_cast<float*>(take(n * fb));
    }
    if (new_xy || S > 1) {
      c.x = reinterpret_cast<float*>(take(n * fb));
      c.y = reinterpret_cast<float*>(take(n * fb));
    }
    return c;
  }

  int max_merge() const { return std::max(1, cfg.max_merge); }   // under mu
  int merge_size = 1;   // the largest max_merge set so far: slot buffers grow to hold it

  size_t held() const {
    size_t b = 0;
    for (const Slot& sl : slots) b += sl.cap;
    return b;
  }

  void drop_graphs(Slot& sl) {
    for (auto& kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
    sl.graphs.clear();
    sl.graph_order.clear();
  }

  // Picks an idle slot for a sweep of `need` bytes and makes its buffer large enough, within
  // the budget: an idle slot that already fits (first one that holds the sweep's captured
  // launch sequence, else the smallest), else the idle slot with the largest buffer grown
  // (to the largest sweep any resident design makes, when that fits the budget), releasing
  // other idle slots' buffers if needed.  -1: wait for a slot to finish.
  int pick_slot(size_t need, const GraphKey& key) {
    int fit = -1, grow = -1;
    bool fit_has = false;
    for (int i = 0; i < (int)slots.size(); ++i) {
      const Slot& sl = slots[i];
      if (sl.busy) continue;
      if (sl.cap >= need) {
        const bool has = sl.graphs.count(key) != 0;
        if (fit < 0 || (has && !fit_has) || (has == fit_has && sl.cap < slots[fit].cap)) {
          fit = i;
          fit_has = has;
        }
      }
      if (grow < 0 || sl.cap > slots[grow].cap) grow = i;
    }
    if (fit >= 0) return fit;
    if (grow < 0) return -1;
    const size_t budget = (size_t)cfg.hbm_budget_bytes;
    size_t target = need;
    for (const Design& d : designs)
      target = std::max(target, request_bytes(d, STA_REQ_FWD_BWD, true, d.can_merge ? merge_size : 1));
    Slot& g = slots[grow];
    auto others = [&] { return held() - g.cap; };
    if (resident + others() + target > budget) target = need;
    if (resident + others() + target > budget) {
      for (Slot& sl : slots)                     // release idle buffers
        if (&sl != &g && !sl.busy && sl.buf) {
          drop_graphs(sl);
          (void)hipFreeAsync(sl.buf, sl.s);
          sl.buf = nullptr;
          sl.cap = 0;
        }
      if (resident + others() + target > budget) return -1;
    }
    const auto t0 = Clock::now();
    drop_graphs(g);
    if (g.buf) (void)hipFreeAsync(g.buf, g.s);
    g.buf = nullptr;
    g.cap = 0;
    hipError_t e = hipMallocFromPoolAsync(&g.buf, target, pool, g.s);
    ++stats.slot_grows;
    stats.grow_ms += ms_between(t0, Clock::now());
    if (e != hipSuccess) {
      g.buf = nullptr;
      return -2;
    }
    g.cap = target;
    return grow;
  }

  // The captured launch sequence of (design, kind, coordinates, gamma, snapshots) over the
  // slot's buffer, captured on first use.  Called by the scheduler thread without the lock:
  // the slot is marked busy, so nothing else touches it, and the design is a copy.  The
  // server alone calls on a resident graph (sta_server_add_design), and only from this
  // thread, so the snapshot count can be set for the capture and put back after it.
  static GraphKey key_of(int design, int kind, bool new_xy, float gamma, int S) {
    uint32_t gb;
    std::memcpy(&gb, &gamma, sizeof(gb));
    return std::make_tuple(design, kind, new_xy || S > 1 ? 1 : 0, gb, S);
  }

  sta_status graph_for(Slot& sl, const Design& d, const Issue& q, hipGraphExec_t* out, int* captured) {
    const GraphKey key = key_of(q.design, q.kind, q.new_xy, q.gamma, q.S);
    auto it = sl.graphs.find(key);
    if (it != sl.graphs.end()) {
      *out = it->second;
      return STA_OK;
    }
    const Carve c = carve(sl.buf, d, q.kind, q.new_xy, q.S);
    const float* x = q.new_xy ? c.x : d.x;
    const float* y = q.new_xy ? c.y : d.y;
    hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    d.g->n_snap = q.S;
    sta_fwd_out fo{c.state, nullptr, nullptr, nullptr, c.sc};
    sta_status st = sta_forward(d.g, x, y, &fo, STA_SMOOTH, q.gamma, cap_stream);
    if (st == STA_OK && q.kind == STA_REQ_FWD_BWD) {
      sta_bwd_out bo{c.ws, nullptr, nullptr, nullptr, nullptr, c.dx, c.dy, 1.0f, nullptr};
      st = sta_backward(d.g, x, y, &fo, &bo, STA_GRAD, q.gamma, cap_stream);
    }
    d.g->n_snap = 1;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap_stream, &graph);
    if (st != STA_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    if (sl.graphs.size() >= kMaxSlotGraphs) {      // bounded cache: evict the oldest capture
      auto old = sl.graphs.find(sl.graph_order.front());
      (void)hipGraphExecDestroy(old->second);
      sl.graphs.erase(old);
      sl.graph_order.pop_front();
    }
    sl.graphs.emplace(key, exec);
    sl.graph_order.push_back(key);
    *out = exec;
    *captured = 1;
    return STA_OK;
  }

  // Issues a sweep on slot sl: coordinates in (snapshot j at offset j * P), the captured
  // launch sequence, results out.  Runs on the scheduler thread without the lock (see
  // graph_for).
  sta_status issue(Slot& sl, const Design& d, const Issue& q, int* captured) {
    const Carve c = carve(sl.buf, d, q.kind, q.new_xy, q.S);
    const size_t P = (size_t)d.P, fb = sizeof(float) * P;
    hipError_t e = hipSuccess;
    hipGraphExec_t exec = nullptr;
    sta_status st = graph_for(sl, d, q, &exec, captured);
    if (st != STA_OK) return st;
    if (q.new_xy) {
      for (size_t j = 0; j < q.m.size() && e == hipSuccess; ++j) {
        const Member& m = q.m[j];
        if (m.hx) {
          if ((e = hipMemcpyAsync(c.x + j * P, m.hx, fb, hipMemcpyHostToDevice, sl.s)) == hipSuccess)
            e = hipMemcpyAsync(c.y + j * P, m.hy, fb, hipMemcpyHostToDevice, sl.s);
        } else if ((e = hipMemcpyAsync(c.x + j * P, d.x, fb, hipMemcpyDeviceToDevice, sl.s)) == hipSuccess) {
          e = hipMemcpyAsync(c.y + j * P, d.y, fb, hipMemcpyDeviceToDevice, sl.s);
        }
      }
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    if ((e = hipGraphLaunch(exec, sl.s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    for (size_t j = 0; j < q.m.size(); ++j) {
      const Member& m = q.m[j];
      if (q.kind == STA_REQ_FWD_BWD) {
        if ((e = hipMemcpyAsync(m.hdx, c.dx + j * P, fb, hipMemcpyDeviceToHost, sl.s)) != hipSuccess ||
            (e = hipMemcpyAsync(m.hdy, c.dy + j * P, fb, hipMemcpyDeviceToHost, sl.s)) != hipSuccess)
          return hip_fail(e, "hipMemcpyAsync");
      }
      if ((e = hipMemcpyAsync(m.hsc, c.sc + 4 * j, 4 * sizeof(double), hipMemcpyDeviceToHost, sl.s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    }
    if ((e = hipEventRecord(sl.done, sl.s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return STA_OK;
  }

  // Queue positions of the requests a sweep headed by the queue's front request takes:
  // itself and the earliest waiting requests of the same design, kind and gamma among the
  // next kMergeWindow, as many as the largest power of two up to max_merge allows.
  static constexpr size_t kMergeWindow = 1024;
  std::vector<size_t> batch_of(const Ticket& head) {
    std::vector<size_t> pos{0};
    if (!designs[head.design].can_merge) return pos;
    const size_t lim = (size_t)max_merge(), end = std::min(queue.size(), kMergeWindow);
    for (size_t i = 1; i < end && pos.size() < lim; ++i) {
      const Ticket& t = tickets[queue[i]];
      if (t.design == head.design && t.kind == head.kind && t.gamma == head.gamma) pos.push_back(i);
    }
    size_t S = 1;
    while (2 * S <= pos.size()) S *= 2;
    pos.resize(S);
    return pos;
  }

  void finish(Ticket& t, TicketState st) {
    t.st = st;
    t.t_done = Clock::now();
    pinned.give(t.hx, sizeof(float) * (size_t)t.P);
    pinned.give(t.hy, sizeof(float) * (size_t)t.P);
    t.hx = t.hy = nullptr;
  }

  void run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool progress = false;
      // Completions.
      int busy = 0;
      for (Slot& sl : slots) {
        if (!sl.busy) continue;
        hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) {
          ++busy;
          continue;
        }
        std::string msg;
        sta_status err = STA_OK;
        if (e != hipSuccess) {
          err = hip_fail(e, "request execution");
          msg = sta_last_error();
        }
        for (uint64_t id : sl.batch) {
          Ticket& t = tickets[id];
          if (e == hipSuccess) {
            finish(t, kDone);
            ++stats.completed;
          } else {
            t.err = err;
            t.msg = msg;
            finish(t, kFailed);
          }
        }
        sl.batch.clear();
        sl.busy = false;
        progress = true;
      }
      if (progress) finished.notify_all();
      // Admissions, in arrival order of the sweeps' first requests.
      while (!queue.empty()) {
        Ticket& head = tickets[queue.front()];
        std::vector<size_t> pos = batch_of(head);
        int k = -1;
        for (;;) {                               // a smaller batch when a larger one cannot fit
          const int S = (int)pos.size();
          k = pick_slot(request_bytes(designs[head.design], head.kind, head.hx != nullptr, S),
                        key_of(head.design, head.kind, head.hx != nullptr, head.gamma, S));
          if (k != -1 || pos.size() == 1) break;
          pos.resize(pos.size() / 2);
        }
        if (k == -1) break;
        if (k == -2) {
          const uint64_t id = queue.front();
          queue.pop_front();
          Ticket& t = tickets[id];
          t.err = fail(STA_E_NOMEM, "slot buffer allocation failed");
          t.msg = sta_last_error();
          finish(t, kFailed);
          finished.notify_all();
          continue;
        }
        std::vector<uint64_t> ids;
        for (size_t i : pos) ids.push_back(queue[i]);
        for (size_t i = pos.size(); i-- > 0;) queue.erase(queue.begin() + (std::ptrdiff_t)pos[i]);
        Slot& sl = slots[k];
        sl.busy = true;
        sl.batch = ids;
        const Ticket& t0 = tickets[ids[0]];
        Issue q{t0.design, t0.kind, t0.gamma, (int)ids.size(), ids.size() > 1 || t0.hx != nullptr, {}};
        const auto now = Clock::now();
        for (uint64_t id : ids) {
          Ticket& t = tickets[id];
          t.t_admit = now;
          t.st = kRunning;
          t.slot = k;
          q.m.push_back(Member{t.hx, t.hy, t.hdx, t.hdy, t.hsc});
        }
        const Design d = designs[t0.design];
        // Capture (first use of a key on this slot) and enqueue without the lock, so that
        // clients can submit and poll meanwhile.
        int captured = 0;
        lk.unlock();
        sta_status st = issue(sl, d, q, &captured);
        std::string msg = st == STA_OK ? std::string() : std::string(sta_last_error());
        lk.lock();
        stats.captures += captured;
        if (captured) stats.capture_ms += ms_between(now, Clock::now());
        if (st != STA_OK) {
          (void)hipStreamSynchronize(sl.s);      // copies already queued still read the staging
          for (uint64_t id : ids) {
            Ticket& tf = tickets[id];
            tf.err = st;
            tf.msg = msg;
            finish(tf, kFailed);
          }
          sl.batch.clear();
          sl.busy = false;
          finished.notify_all();
          continue;
        }
        ++stats.sweeps;
        if (ids.size() > 1) stats.merged += (int64_t)ids.size();
        ++busy;
        progress = true;
      }
      if (stop && busy == 0) break;
      if (!progress) {
        if (busy > 0)
          wake.wait_for(lk, std::chrono::microseconds(20));
        else
          wake.wait(lk, [&] { return stop || !queue.empty(); });
      }
    }
  }
};

extern "C" {

sta_status sta_server_create(const sta_server_config* cfg, sta_server** out) {
  if (!cfg || !out) return fail(STA_E_INVALID, "NULL argument");
  if (cfg->hbm_budget_bytes <= 0 || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->queue_capacity < 1)
    return fail(STA_E_INVALID, "server configuration out of range");
  if (cfg->max_merge < 0 || cfg->max_merge > 64 || (cfg->max_merge & (cfg->max_merge - 1)) != 0)
    return fail(STA_E_INVALID, "max_merge must be 0 or a power of two up to 64");
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  int pools = 0;
  e = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  if (!pools) return fail(STA_E_DEVICE, "device has no stream-ordered memory pools");
  sta_server* s = nullptr;
  try {
    s = new sta_server;
  } catch (const std::bad_alloc&) {
    return fail(STA_E_NOMEM, "host allocation failed");
  }
  s->cfg = *cfg;
  s->merge_size = std::max(1, cfg->max_merge);
  s->device = dev;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  sta_status st = STA_OK;
  if ((e = hipMemPoolCreate(&s->pool, &props)) != hipSuccess) st = hip_fail(e, "hipMemPoolCreate");
  if (st == STA_OK) {
    uint64_t keep = UINT64_MAX;   // freed blocks stay in the pool for the next request
    if ((e = hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &keep)) != hipSuccess)
      st = hip_fail(e, "hipMemPoolSetAttribute");
  }
  if (st == STA_OK && (e = hipStreamCreateWithFlags(&s->setup_stream, hipStreamNonBlocking)) != hipSuccess)
    st = hip_fail(e, "hipStreamCreateWithFlags");
  if (st == STA_OK && (e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    st = hip_fail(e, "hipStreamCreateWithFlags");
  s->slots.resize(cfg->max_slots);
  for (Slot& sl : s->slots) {
    if (st != STA_OK) break;
    if ((e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
      st = hip_fail(e, "slot stream");
  }
  if (st == STA_OK) {
    try {
      s->worker = std::thread([s] { s->run(); });
    } catch (...) {
      st = fail(STA_E_NOMEM, "cannot start the scheduler thread");
    }
  }
  if (st != STA_OK) {
    sta_server_destroy(s);
    return st;
  }
  *out = s;
  return STA_OK;
}

sta_status sta_server_add_design(sta_server* s, sta_graph* g, const float* x, const float* y, int32_t* id) {
  if (!s || !g || !x || !y || !id) return fail(STA_E_INVALID, "NULL argument");
  if (!g->levelized) return fail(STA_E_STATE, "graph is not levelized");
  if (g->n_snap != 1) return fail(STA_E_INVALID, "served graphs sweep one snapshot per request");
  int cur = -1;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(s->device);
  struct Restore {
    int d;
    ~Restore() {
      if (d >= 0) (void)hipSetDevice(d);
    }
  } restore{cur};
  sta_status st = sta_graph_upload(g);
  if (st != STA_OK) return st;
  const size_t fb = sizeof(float) * (size_t)g->P;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->resident + g->dev.bytes + 2 * fb > (size_t)s->cfg.hbm_budget_bytes)
      return fail(STA_E_NOMEM, "design does not fit the server's memory budget");
  }
  Design d;
  d.g = g;
  d.P = g->P;
  d.state_bytes = g->state.total;
  d.work_bytes = g->work.total;
  d.can_merge = !g->snap_inner && g->sched_cfg.level_scheme == STA_LEVEL_GROUPS && g->n_designs == 1 &&
                g->state.total <= (size_t)INT32_MAX;     // as sta_set_snapshots requires
  hipError_t e;
  if ((e = hipMalloc(&d.x, std::max<size_t>(fb, 4))) != hipSuccess) return hip_fail(e, "hipMalloc");
  if ((e = hipMalloc(&d.y, std::max<size_t>(fb, 4))) != hipSuccess) {
    (void)hipFree(d.x);
    return hip_fail(e, "hipMalloc");
  }
  if ((e = hipMemcpyAsync(d.x, x, fb, hipMemcpyHostToDevice, s->setup_stream)) != hipSuccess ||
      (e = hipMemcpyAsync(d.y, y, fb, hipMemcpyHostToDevice, s->setup_stream)) != hipSuccess ||
      (e = hipStreamSynchronize(s->setup_stream)) != hipSuccess) {
    (void)hipFree(d.x);
    (void)hipFree(d.y);
    return hip_fail(e, "coordinate upload");
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->resident += g->dev.bytes + 2 * fb;
  s->designs.push_back(d);
  *id = (int32_t)s->designs.size() - 1;
  return STA_OK;
}

sta_status sta_submit(sta_server* s, const sta_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return fail(STA_E_INVALID, "NULL argument");
  if ((r->x == nullptr) != (r->y == nullptr)) return fail(STA_E_INVALID, "give both x and y, or neither");
  if (r->kind != STA_REQ_FWD && r->kind != STA_REQ_FWD_BWD) return fail(STA_E_INVALID, "unknown request kind");
  if (!(r->gamma_ps > 0.f && std::isfinite(r->gamma_ps))) return fail(STA_E_INVALID, "gamma must be positive");
  Ticket t;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->design < 0 || r->design >= (int)s->designs.size()) return fail(STA_E_INVALID, "unknown design");
    const Design& d = s->designs[r->design];
    t.need = s->request_bytes(d, r->kind, r->x != nullptr);
    t.P = d.P;
    if (s->resident + t.need > (size_t)s->cfg.hbm_budget_bytes)
      return fail(STA_E_NOMEM, "request can never fit the server's memory budget");
    if ((int)s->queue.size() >= s->cfg.queue_capacity) return fail(STA_E_BUSY, "admission queue is full");
  }
  t.design = r->design;
  t.kind = r->kind;
  t.gamma = r->gamma_ps;
  t.t_submit = Clock::now();
  const size_t fb = sizeof(float) * (size_t)t.P;
  bool ok = true;
  if (r->x) {
    t.hx = static_cast<float*>(s->pinned.take(fb));
    t.hy = static_cast<float*>(s->pinned.take(fb));
    ok = t.hx && t.hy;
    if (ok) {
      std::memcpy(t.hx, r->x, fb);
      std::memcpy(t.hy, r->y, fb);
    }
  }
  t.hsc = static_cast<double*>(s->pinned.take(4 * sizeof(double)));
  ok = ok && t.hsc;
  if (ok && t.kind == STA_REQ_FWD_BWD) {
    t.hdx = static_cast<float*>(s->pinned.take(fb));
    t.hdy = static_cast<float*>(s->pinned.take(fb));
    ok = t.hdx && t.hdy;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (!ok) {
    s->pinned.give(t.hx, fb);
    s->pinned.give(t.hy, fb);
    s->pinned.give(t.hsc, 4 * sizeof(double));
    s->pinned.give(t.hdx, fb);
    s->pinned.give(t.hdy, fb);
    return fail(STA_E_NOMEM, "pinned host allocation failed");
  }
  const uint64_t id = s->next_ticket++;
  s->tickets.emplace(id, std::move(t));
  s->queue.push_back(id);
  *ticket = id;
  s->wake.notify_one();
  return STA_OK;
}

static sta_status fill_result(sta_server* s, uint64_t ticket, sta_result* r) {
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(STA_E_UNKNOWN_TICKET, "unknown ticket");
  const Ticket& t = it->second;
  if (t.st == kQueued || t.st == kRunning) return STA_PENDING;
  if (t.st == kFailed) return fail(t.err, t.msg);
  if (r) {
    r->kind = t.kind;
    r->n_pins = t.P;
    std::memcpy(r->scalars, t.hsc, sizeof(r->scalars));
    r->dx = t.hdx;
    r->dy = t.hdy;
    r->queue_ms = ms_between(t.t_submit, t.t_admit);
    r->latency_ms = ms_between(t.t_submit, t.t_done);
  }
  return STA_OK;
}

sta_status sta_server_set_max_merge(sta_server* s, int32_t max_merge) {
  if (!s) return fail(STA_E_INVALID, "NULL argument");
  if (max_merge < 0 || max_merge > 64 || (max_merge & (max_merge - 1)) != 0)
    return fail(STA_E_INVALID, "max_merge must be 0 or a power of two up to 64");
  std::lock_guard<std::mutex> lk(s->mu);
  s->cfg.max_merge = max_merge;
  s->merge_size = std::max(s->merge_size, max_merge);
  return STA_OK;
}

sta_status sta_server_stats_get(sta_server* s, sta_server_stats* out) {
  if (!s || !out) return fail(STA_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  s->pinned.counts(&out->pinned_allocs, &out->pinned_ms);
  return STA_OK;
}

sta_status sta_poll(sta_server* s, uint64_t ticket, sta_result* r) {
  if (!s) return fail(STA_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  return fill_result(s, ticket, r);
}

sta_status sta_wait(sta_server* s, uint64_t ticket, sta_result* r) {
  if (!s) return fail(STA_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    sta_status st = fill_result(s, ticket, r);
    if (st != STA_PENDING) return st;
    s->finished.wait(lk);
  }
}

sta_status sta_release(sta_server* s, uint64_t ticket) {
  if (!s) return fail(STA_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(STA_E_UNKNOWN_TICKET, "unknown ticket");
  Ticket& t = it->second;
  if (t.st == kRunning) return fail(STA_E_BUSY, "request is on the device");
  if (t.st == kQueued) s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
  const size_t fb = sizeof(float) * (size_t)t.P;
  s->pinned.give(t.hx, fb);
  s->pinned.give(t.hy, fb);
  s->pinned.give(t.hsc, 4 * sizeof(double));
  s->pinned.give(t.hdx, fb);
  s->pinned.give(t.hdy, fb);
  s->tickets.erase(it);
  return STA_OK;
}

void sta_server_destroy(sta_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->wake.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Slot& sl : s->slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    s->drop_graphs(sl);
    if (sl.buf) {
      (void)hipFreeAsync(sl.buf, sl.s);
      (void)hipStreamSynchronize(sl.s);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.s) (void)hipStreamDestroy(sl.s);
  }
  for (auto& kv : s->tickets) {
    Ticket& t = kv.second;
    const size_t fb = sizeof(float) * (size_t)t.P;
    s->pinned.give(t.hx, fb);
    s->pinned.give(t.hy, fb);
    s->pinned.give(t.hsc, 4 * sizeof(double));
    s->pinned.give(t.hdx, fb);
    s->pinned.give(t.hdy, fb);
  }
  for (Design& d : s->designs) {
    (void)hipFree(d.x);
    (void)hipFree(d.y);
  }
  if (s->setup_stream) (void)hipStreamDestroy(s->setup_stream);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->pool) (void)hipMemPoolDestroy(s->pool);
  delete s;
}

}  // extern "C"
