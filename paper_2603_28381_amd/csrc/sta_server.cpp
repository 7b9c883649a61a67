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
    if (hipHostMalloc(&p, std::max<size_t>(bytes, 1), hipHostMallocDefault) != hipSuccess) return nullptr;
    return p;
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
};

struct Design {
  sta_graph* g = nullptr;
  int P = 0;
  float* x = nullptr;   // resident coordinates (device, original order)
  float* y = nullptr;
  size_t state_bytes = 0, work_bytes = 0;
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

// A slot runs one request at a time on its own stream, in a device buffer it keeps between
// requests, with the launch sequence of each (design, kind, coordinates) captured once into
// a hipGraph over that buffer and replayed afterwards.
using GraphKey = std::tuple<int, int, int, uint32_t>;   // (design, kind, new x/y, gamma bits)
constexpr size_t kMaxSlotGraphs = 64;   // captured sequences kept per slot; the oldest goes first

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  uint64_t ticket = 0;
  bool busy = false;
  void* buf = nullptr;          // from the server's pool
  size_t cap = 0;
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::deque<GraphKey> graph_order;   // capture order, for eviction
};

// What issuing a request needs, copied out of the ticket and the design table so that the
// scheduler can capture and enqueue without holding the server's lock.
struct Issue {
  int design, kind;
  float gamma;
  const float *hx, *hy;
  float *hdx, *hdy;
  double* hsc;
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

  size_t request_bytes(const Design& d, int kind, bool new_xy) const {
    size_t b = align256(d.state_bytes) + align256(4 * sizeof(double));
    if (kind == STA_REQ_FWD_BWD) b += align256(d.work_bytes) + 2 * align256(sizeof(float) * (size_t)d.P);
    if (new_xy) b += 2 * align256(sizeof(float) * (size_t)d.P);
    return b;
  }

  static Carve carve(void* base, const Design& d, int kind, bool new_xy) {
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) {
      char* r = p;
      p += align256(bytes);
      return r;
    };
    const size_t fb = sizeof(float) * (size_t)d.P;
    Carve c{};
    c.state = take(d.state_bytes);
    c.sc = reinterpret_cast<double*>(take(4 * sizeof(double)));
    if (kind == STA_REQ_FWD_BWD) {
      c.ws = take(d.work_bytes);
      c.dx = reinterpret_cast<float*>(take(fb));
      c.dy = reinterpret_cast<float*>(take(fb));
    }
    if (new_xy) {
      c.x = reinterpret_cast<float*>(take(fb));
      c.y = reinterpret_cast<float*>(take(fb));
    }
    return c;
  }

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

  // Picks an idle slot for a request of `need` bytes and makes its buffer large enough,
  // within the budget: an idle slot that already fits, else the idle slot with the largest
  // buffer grown (to the largest request any resident design makes, when that fits the
  // budget), releasing other idle slots' buffers if needed.  -1: wait for a slot to finish.
  int pick_slot(size_t need) {
    int fit = -1, grow = -1;
    for (int i = 0; i < (int)slots.size(); ++i) {
      const Slot& sl = slots[i];
      if (sl.busy) continue;
      if (sl.cap >= need && (fit < 0 || sl.cap < slots[fit].cap)) fit = i;
      if (grow < 0 || sl.cap > slots[grow].cap) grow = i;
    }
    if (fit >= 0) return fit;
    if (grow < 0) return -1;
    const size_t budget = (size_t)cfg.hbm_budget_bytes;
    size_t target = need;
    for (const Design& d : designs) target = std::max(target, request_bytes(d, STA_REQ_FWD_BWD, true));
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
    drop_graphs(g);
    if (g.buf) (void)hipFreeAsync(g.buf, g.s);
    g.buf = nullptr;
    g.cap = 0;
    hipError_t e = hipMallocFromPoolAsync(&g.buf, target, pool, g.s);
    if (e != hipSuccess) {
      g.buf = nullptr;
      return -2;
    }
    g.cap = target;
    return grow;
  }

  // The captured launch sequence of (design, kind, coordinates, gamma) over the slot's
  // buffer, captured on first use.  Called by the scheduler thread without the lock: the
  // slot is marked busy, so nothing else touches it, and the design is a copy.
  sta_status graph_for(Slot& sl, const Design& d, const Issue& q, hipGraphExec_t* out, int* captured) {
    uint32_t gb;
    std::memcpy(&gb, &q.gamma, sizeof(gb));
    const GraphKey key = std::make_tuple(q.design, q.kind, q.hx ? 1 : 0, gb);
    auto it = sl.graphs.find(key);
    if (it != sl.graphs.end()) {
      *out = it->second;
      return STA_OK;
    }
    const Carve c = carve(sl.buf, d, q.kind, q.hx != nullptr);
    const float* x = q.hx ? c.x : d.x;
    const float* y = q.hx ? c.y : d.y;
    hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    sta_fwd_out fo{c.state, nullptr, nullptr, nullptr, c.sc};
    sta_status st = sta_forward(d.g, x, y, &fo, STA_SMOOTH, q.gamma, cap_stream);
    if (st == STA_OK && q.kind == STA_REQ_FWD_BWD) {
      sta_bwd_out bo{c.ws, nullptr, nullptr, nullptr, nullptr, c.dx, c.dy, 1.0f, nullptr};
      st = sta_backward(d.g, x, y, &fo, &bo, STA_GRAD, q.gamma, cap_stream);
    }
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

  // Issues a request on slot sl: coordinates in, the captured sweeps, results out.  Runs
  // on the scheduler thread without the lock (see graph_for).
  sta_status issue(Slot& sl, const Design& d, const Issue& q, int* captured) {
    const Carve c = carve(sl.buf, d, q.kind, q.hx != nullptr);
    const size_t fb = sizeof(float) * (size_t)d.P;
    hipError_t e;
    hipGraphExec_t exec = nullptr;
    sta_status st = graph_for(sl, d, q, &exec, captured);
    if (st != STA_OK) return st;
    if (q.hx) {
      if ((e = hipMemcpyAsync(c.x, q.hx, fb, hipMemcpyHostToDevice, sl.s)) != hipSuccess ||
          (e = hipMemcpyAsync(c.y, q.hy, fb, hipMemcpyHostToDevice, sl.s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    }
    if ((e = hipGraphLaunch(exec, sl.s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if (q.kind == STA_REQ_FWD_BWD) {
      if ((e = hipMemcpyAsync(q.hdx, c.dx, fb, hipMemcpyDeviceToHost, sl.s)) != hipSuccess ||
          (e = hipMemcpyAsync(q.hdy, c.dy, fb, hipMemcpyDeviceToHost, sl.s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    }
    if ((e = hipMemcpyAsync(q.hsc, c.sc, 4 * sizeof(double), hipMemcpyDeviceToHost, sl.s)) != hipSuccess)
      return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipEventRecord(sl.done, sl.s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return STA_OK;
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
        Ticket& t = tickets[sl.ticket];
        if (e == hipSuccess) {
          finish(t, kDone);
          ++stats.completed;
        } else {
          t.err = hip_fail(e, "request execution");
          t.msg = sta_last_error();
          finish(t, kFailed);
        }
        sl.busy = false;
        progress = true;
      }
      if (progress) finished.notify_all();
      // Admissions, in arrival order.
      while (!queue.empty()) {
        const uint64_t id = queue.front();
        Ticket& t = tickets[id];
        const int k = pick_slot(t.need);
        if (k == -1) break;
        if (k == -2) {
          queue.pop_front();
          t.err = fail(STA_E_NOMEM, "slot buffer allocation failed");
          t.msg = sta_last_error();
          finish(t, kFailed);
          finished.notify_all();
          continue;
        }
        queue.pop_front();
        t.t_admit = Clock::now();
        t.st = kRunning;
        t.slot = k;
        Slot& sl = slots[k];
        sl.busy = true;
        sl.ticket = id;
        const Issue q{t.design, t.kind, t.gamma, t.hx, t.hy, t.hdx, t.hdy, t.hsc};
        const Design d = designs[t.design];
        // Capture (first use of a key on this slot) and enqueue without the lock, so that
        // clients can submit and poll meanwhile.
        int captured = 0;
        const auto c0 = Clock::now();
        lk.unlock();
        sta_status st = issue(sl, d, q, &captured);
        std::string msg = st == STA_OK ? std::string() : std::string(sta_last_error());
        lk.lock();
        stats.captures += captured;
        if (captured) stats.capture_ms += ms_between(c0, Clock::now());
        if (st != STA_OK) {
          Ticket& tf = tickets[id];
          tf.err = st;
          tf.msg = msg;
          finish(tf, kFailed);
          sl.busy = false;
          finished.notify_all();
          continue;
        }
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

sta_status sta_server_stats_get(sta_server* s, sta_server_stats* out) {
  if (!s || !out) return fail(STA_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
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
