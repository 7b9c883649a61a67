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
  size_t need = 0;       // device bytes while on the device
  void* dmem = nullptr;
  int slot = -1;
  Clock::time_point t_submit, t_admit, t_done;
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  uint64_t ticket = 0;
  bool busy = false;
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
  size_t in_flight = 0;       // bytes of requests on the device
  std::mutex mu;
  std::condition_variable wake;       // scheduler: new work or stop
  std::condition_variable finished;   // waiters: a ticket finished
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  PinnedPool pinned;

  size_t request_bytes(const Design& d, int kind, bool new_xy) const {
    size_t b = align256(d.state_bytes) + align256(4 * sizeof(double));
    if (kind == STA_REQ_FWD_BWD) b += align256(d.work_bytes) + 2 * align256(sizeof(float) * (size_t)d.P);
    if (new_xy) b += 2 * align256(sizeof(float) * (size_t)d.P);
    return b;
  }

  // Issues a request's copies and sweeps on slot k's stream.  Called with mu held.  On a
  // failure the request's memory goes back to the pool in stream order.
  sta_status launch(uint64_t id, Ticket& t, int k) {
    Slot& sl = slots[k];
    hipError_t e = hipMallocFromPoolAsync(&t.dmem, t.need, pool, sl.s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocFromPoolAsync");
    sta_status st = enqueue(t, sl);
    if (st != STA_OK) {
      (void)hipFreeAsync(t.dmem, sl.s);
      return st;
    }
    if ((e = hipFreeAsync(t.dmem, sl.s)) != hipSuccess) return hip_fail(e, "hipFreeAsync");
    if ((e = hipEventRecord(sl.done, sl.s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    sl.busy = true;
    sl.ticket = id;
    t.slot = k;
    return STA_OK;
  }

  sta_status enqueue(Ticket& t, Slot& sl) {
    const Design& d = designs[t.design];
    hipError_t e;
    char* p = static_cast<char*>(t.dmem);
    auto carve = [&](size_t bytes) {
      char* r = p;
      p += align256(bytes);
      return r;
    };
    void* state = carve(d.state_bytes);
    double* sc = reinterpret_cast<double*>(carve(4 * sizeof(double)));
    const size_t fb = sizeof(float) * (size_t)d.P;
    const float* x = d.x;
    const float* y = d.y;
    void* ws = nullptr;
    float *dx = nullptr, *dy = nullptr;
    if (t.kind == STA_REQ_FWD_BWD) {
      ws = carve(d.work_bytes);
      dx = reinterpret_cast<float*>(carve(fb));
      dy = reinterpret_cast<float*>(carve(fb));
    }
    if (t.hx) {
      float* nx = reinterpret_cast<float*>(carve(fb));
      float* ny = reinterpret_cast<float*>(carve(fb));
      if ((e = hipMemcpyAsync(nx, t.hx, fb, hipMemcpyHostToDevice, sl.s)) != hipSuccess ||
          (e = hipMemcpyAsync(ny, t.hy, fb, hipMemcpyHostToDevice, sl.s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
      x = nx;
      y = ny;
    }
    sta_fwd_out fo{state, nullptr, nullptr, nullptr, sc};
    sta_status st = sta_forward(d.g, x, y, &fo, STA_SMOOTH, t.gamma, sl.s);
    if (st != STA_OK) return st;
    if (t.kind == STA_REQ_FWD_BWD) {
      sta_bwd_out bo{ws, nullptr, nullptr, nullptr, nullptr, dx, dy, 1.0f, nullptr};
      st = sta_backward(d.g, x, y, &fo, &bo, STA_GRAD, t.gamma, sl.s);
      if (st != STA_OK) return st;
      if ((e = hipMemcpyAsync(t.hdx, dx, fb, hipMemcpyDeviceToHost, sl.s)) != hipSuccess ||
          (e = hipMemcpyAsync(t.hdy, dy, fb, hipMemcpyDeviceToHost, sl.s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    }
    if ((e = hipMemcpyAsync(t.hsc, sc, 4 * sizeof(double), hipMemcpyDeviceToHost, sl.s)) != hipSuccess)
      return hip_fail(e, "hipMemcpyAsync");
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
        } else {
          t.err = hip_fail(e, "request execution");
          t.msg = sta_last_error();
          finish(t, kFailed);
        }
        in_flight -= t.need;
        sl.busy = false;
        progress = true;
      }
      if (progress) finished.notify_all();
      // Admissions, in arrival order.
      while (!queue.empty()) {
        int k = -1;
        for (int i = 0; i < (int)slots.size(); ++i)
          if (!slots[i].busy) {
            k = i;
            break;
          }
        if (k < 0) break;
        const uint64_t id = queue.front();
        Ticket& t = tickets[id];
        if (resident + in_flight + t.need > (size_t)cfg.hbm_budget_bytes) break;
        queue.pop_front();
        t.t_admit = Clock::now();
        t.st = kRunning;
        sta_status st = launch(id, t, k);
        if (st != STA_OK) {
          t.err = st;
          t.msg = sta_last_error();
          finish(t, kFailed);
          finished.notify_all();
          continue;
        }
        in_flight += t.need;
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
  if (s->pool) (void)hipMemPoolDestroy(s->pool);
  delete s;
}

}  // extern "C"
