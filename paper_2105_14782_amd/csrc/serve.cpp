// exohip serving engine: memory-admitted continuous batching on HIP streams.
// C ABI in include/exohip_serve.h.
#include <hip/hip_runtime.h>

#include <time.h>

#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/exohip_serve.h"
#include "exo_host.h"

using namespace exo;

namespace {

// Seconds on CLOCK_MONOTONIC: the clock callers state arrival times in.
double mono_now() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

// A request waiting for memory at the head of the queue lets at most this
// many later requests that fit be admitted before it; then admission waits
// for it (no starvation of large requests).
constexpr int kMaxBypass = 8;
// How far past a waiting head the dispatcher looks for a request that fits.
constexpr size_t kBypassWindow = 64;

struct Request {
  int64_t id = 0;
  std::vector<double> P, logx, T;
  std::vector<int32_t> species;
  exo_atmos atm{};
  exo_response resp{};
  bool has_resp = false;
  int precision = 0;
  void* flux = nullptr;
  size_t bytes = 0;
  size_t region = 0;
  int slot = -1;
  int bypassed = 0;   // later requests admitted while this one waited at the head for memory
  int passed = 0;     // shortest first: later requests admitted ahead of this one
  double work = 0;    // shortest first: line x point x layer evaluations
  double t_arrival = 0, t_admit = 0, t_done = 0;   // CLOCK_MONOTONIC seconds
  int status = EXO_OK;
  std::string msg;
  bool done = false;
};

struct Slot {
  hipStream_t st = nullptr;
  Workspace ws;
  bool busy = false;
};

// First-fit allocator of contiguous regions of the memory budget.
class Regions {
 public:
  void init(size_t cap) {
    free_.clear();
    free_[0] = cap;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, o2 = it->first + n;
        free_.erase(it);
        if (rest) free_[o2] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

constexpr size_t kAlign = 256;

}  // namespace

struct exo_server {
  exo_ctx* ctx = nullptr;
  int device = 0;
  std::vector<std::unique_ptr<Slot>> slots;
  char* arena = nullptr;
  size_t cap = 0, in_use = 0, peak = 0;
  Regions regions;
  std::mutex mu;
  std::condition_variable cv;       // wakes the dispatcher
  std::condition_variable done_cv;  // wakes waiters
  std::deque<std::shared_ptr<Request>> queue;
  std::map<int64_t, std::shared_ptr<Request>> live;  // submitted, not yet waited for
  std::vector<Request*> finished;                   // reported by stream callbacks
  int64_t next_id = 1;
  int64_t submitted = 0, admitted = 0, completed = 0, failed = 0, rejected = 0, in_flight = 0;
  int64_t peak_in_flight = 0, bypasses = 0;
  int policy = EXO_SERVE_FIFO;
  int max_passes = 16;
  bool stop = false;
  std::thread dispatcher;
};

namespace {

struct CallbackArg {
  exo_server* srv;
  Request* req;
};

// Runs on a HIP runtime thread when the request's last kernel has finished;
// no HIP calls here, only bookkeeping.
void on_stream_done(void* p) {
  CallbackArg* a = static_cast<CallbackArg*>(p);
  {
    std::lock_guard<std::mutex> g(a->srv->mu);
    a->req->t_done = mono_now();
    a->srv->finished.push_back(a->req);
  }
  a->srv->cv.notify_all();
  delete a;
}

// The request admission prefers: the queue head (FIFO), or (shortest first)
// the earliest request of the look-ahead window that has been passed over
// max_passes times, else the window's smallest request (earliest on ties).
std::deque<std::shared_ptr<Request>>::iterator preferred(exo_server* s) {
  auto it = s->queue.begin();
  if (s->policy == EXO_SERVE_FIFO) return it;
  const auto end = s->queue.size() > kBypassWindow ? s->queue.begin() + kBypassWindow : s->queue.end();
  auto best = it;
  for (auto q = it; q != end; ++q) {
    if ((*q)->passed >= s->max_passes) return q;
    if ((*q)->work < (*best)->work) best = q;
  }
  return best;
}

int free_slot(exo_server* s) {
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (!s->slots[i]->busy) return (int)i;
  return -1;
}

void run_dispatcher(exo_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv.wait(lk, [&] {
      if (s->stop || !s->finished.empty()) return true;
      if (s->queue.empty() || free_slot(s) < 0) return false;
      return true;  // try admission (may still lack memory; re-waits below)
    });
    // retire finished requests: free their slot and memory region
    bool retired = false;
    for (Request* r : s->finished) {
      s->slots[r->slot]->busy = false;
      s->regions.release(r->region, r->bytes);
      s->in_use -= r->bytes;
      --s->in_flight;
      if (r->status == EXO_OK) ++s->completed;
      else ++s->failed;
      r->done = true;
      retired = true;
    }
    s->finished.clear();
    if (retired) s->done_cv.notify_all();
    if (s->stop && s->queue.empty() && s->in_flight == 0) break;
    // admit while a slot and a memory region are free, the preferred request
    // first (the head in arrival order, or by the shortest-first rule); one
    // that waits for memory lets up to kMaxBypass other requests that fit go
    // first (looking kBypassWindow requests ahead)
    bool admitted_any = false;
    while (!s->queue.empty()) {
      const int si = free_slot(s);
      if (si < 0) break;
      size_t off;
      auto pick = preferred(s);
      if (!s->regions.alloc((*pick)->bytes, &off)) {
        Request* head = pick->get();
        if (head->bypassed >= kMaxBypass) break;  // wait for memory
        const auto end = s->queue.size() > kBypassWindow ? s->queue.begin() + kBypassWindow : s->queue.end();
        for (pick = s->queue.begin(); pick != end; ++pick)
          if (pick->get() != head && s->regions.alloc((*pick)->bytes, &off)) break;
        if (pick == end) break;  // nothing fits: wait for memory
        ++head->bypassed;
        ++s->bypasses;
      }
      // every earlier arrival still queued has been passed over once more
      for (auto q = s->queue.begin(); q != pick; ++q) ++(*q)->passed;
      std::shared_ptr<Request> r = *pick;
      s->queue.erase(pick);
      r->region = off;
      r->slot = si;
      r->t_admit = mono_now();
      Slot& sl = *s->slots[si];
      sl.busy = true;
      s->in_use += r->bytes;
      if (s->in_use > s->peak) s->peak = s->in_use;
      ++s->admitted;
      ++s->in_flight;
      if (s->in_flight > s->peak_in_flight) s->peak_in_flight = s->in_flight;
      admitted_any = true;
      lk.unlock();
      sl.ws.bind_arena(s->arena + off, r->bytes);
      int rc = emission_impl(s->ctx, sl.ws, &r->atm, r->has_resp ? &r->resp : nullptr, r->precision,
                             r->flux, sl.st);
      if (rc != EXO_OK) {
        r->status = rc;
        r->msg = exo_last_error();
      }
      CallbackArg* cb = new CallbackArg{s, r.get()};
      if (hipLaunchHostFunc(sl.st, on_stream_done, cb) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(sl.st);
        on_stream_done(cb);
      }
      lk.lock();
    }
    if (!admitted_any && !s->stop && s->finished.empty() && !s->queue.empty()) {
      // head waits for memory or a slot: sleep until a request finishes
      s->cv.wait(lk, [&] { return s->stop || !s->finished.empty(); });
    }
  }
}

}  // namespace

extern "C" int exo_server_create(exo_ctx* ctx, int n_streams, size_t budget, exo_server** out) {
  if (!ctx || !out) return set_err(EXO_EINVAL, "NULL argument");
  *out = nullptr;
  if (n_streams < 1 || n_streams > 16) return set_err(EXO_EINVAL, "n_streams must be in 1..16");
  if (budget < (size_t(1) << 20)) return set_err(EXO_EINVAL, "memory budget below 1 MiB");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(EXO_EDEVICE, "hipSetDevice failed");
  auto* s = new exo_server();
  s->ctx = ctx;
  s->device = ctx->device;
  s->cap = budget & ~(kAlign - 1);
  if (fail_alloc_hook() || hipMalloc((void**)&s->arena, s->cap) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return set_err(EXO_ENOMEM, "cannot allocate the %zu-byte serving budget", budget);
  }
  s->regions.init(s->cap);
  for (int i = 0; i < n_streams; ++i) {
    auto sl = std::make_unique<Slot>();
    if (hipStreamCreateWithFlags(&sl->st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      for (auto& x : s->slots) (void)hipStreamDestroy(x->st);
      (void)hipFree(s->arena);
      delete s;
      return set_err(EXO_EDEVICE, "hipStreamCreate failed");
    }
    s->slots.push_back(std::move(sl));
  }
  s->dispatcher = std::thread(run_dispatcher, s);
  *out = s;
  return EXO_OK;
}

extern "C" int exo_server_set_policy(exo_server* s, int policy, int max_passes) {
  if (!s) return set_err(EXO_EINVAL, "NULL server");
  if (policy != EXO_SERVE_FIFO && policy != EXO_SERVE_SHORTEST_FIRST)
    return set_err(EXO_EINVAL, "unknown admission policy %d", policy);
  if (max_passes < 1 || max_passes > (1 << 20)) return set_err(EXO_EINVAL, "max_passes must be in 1..2^20");
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->policy = policy;
    s->max_passes = max_passes;
  }
  s->cv.notify_all();
  return EXO_OK;
}

extern "C" int exo_server_destroy(exo_server* s) {
  if (!s) return EXO_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  s->dispatcher.join();
  (void)hipSetDevice(s->device);
  for (auto& sl : s->slots) {
    (void)hipStreamSynchronize(sl->st);
    sl->ws.bind_arena(nullptr, 0);
    sl->ws.release();
    (void)hipStreamDestroy(sl->st);
  }
  (void)hipFree(s->arena);
  delete s;
  return EXO_OK;
}

extern "C" size_t exo_workspace_bytes(exo_ctx* ctx, const exo_atmos* a, const exo_response* r,
                                      int precision) {
  if (!ctx || !a || (precision != EXO_FP32_KAHAN && precision != EXO_FP64)) return 0;
  return estimate_workspace(ctx, a, r, precision == EXO_FP64, false);
}

extern "C" int exo_server_submit(exo_server* s, const exo_atmos* a, const exo_response* r,
                                 int precision, void* flux, double arrival_s, int64_t* ticket) {
  if (!s || !a || !ticket) return set_err(EXO_EINVAL, "NULL argument");
  if (!flux) return set_err(EXO_EINVAL, "flux_dev is NULL");
  if (precision != EXO_FP32_KAHAN && precision != EXO_FP64) return set_err(EXO_EINVAL, "bad precision");
  if (!std::isfinite(arrival_s)) return set_err(EXO_EINVAL, "arrival time must be finite");
  int64_t gb, gl;
  int rc;
  if ((rc = validate_atmos(s->ctx, a, &gb, &gl))) return rc;
  if (r) {
    RespDev R{};
    if ((rc = prepare_response(s->ctx, r, gl, &R))) return rc;
  }
  const size_t bytes = estimate_workspace(s->ctx, a, r, precision == EXO_FP64, false);
  if (bytes == 0) return set_err(EXO_EINVAL, "invalid request");
  auto q = std::make_shared<Request>();
  q->bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
  for (int m = 0; m < a->n_species; ++m) q->work += (double)s->ctx->sp[a->species[m]].n;
  q->work *= (double)gl * (double)a->n_layers;
  if (q->bytes > s->cap) {
    std::lock_guard<std::mutex> g(s->mu);
    ++s->rejected;
    return set_err(EXO_ENOMEM, "request needs %zu bytes, the serving budget is %zu", q->bytes, s->cap);
  }
  q->P.assign(a->P_bar, a->P_bar + a->n_layers);
  q->logx.assign(a->log10_mmr, a->log10_mmr + a->n_species);
  q->species.assign(a->species, a->species + a->n_species);
  q->atm = *a;
  q->atm.P_bar = q->P.data();
  q->atm.log10_mmr = q->logx.data();
  q->atm.species = q->species.data();
  if (a->T_layers) {
    q->T.assign(a->T_layers, a->T_layers + a->n_layers);
    q->atm.T_layers = q->T.data();
  }
  if (r) {
    q->resp = *r;
    q->has_resp = true;
  }
  q->precision = precision;
  q->flux = flux;
  const double now = mono_now();
  q->t_arrival = arrival_s > 0 && arrival_s <= now ? arrival_s : now;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return set_err(EXO_EINVAL, "server is shutting down");
    q->id = s->next_id++;
    s->live[q->id] = q;
    s->queue.push_back(q);
    ++s->submitted;
    *ticket = q->id;
  }
  s->cv.notify_all();
  return EXO_OK;
}

extern "C" int exo_server_wait(exo_server* s, int64_t ticket, double timeout_s, double* latency_s,
                               double* queue_s) {
  if (!s) return set_err(EXO_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->live.find(ticket);
  if (it == s->live.end()) return set_err(EXO_EINVAL, "unknown ticket %lld", (long long)ticket);
  std::shared_ptr<Request> r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_s < 0) s->done_cv.wait(lk, ready);
  else if (!s->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
    return set_err(EXO_EINVAL, "timeout waiting for ticket %lld", (long long)ticket);
  s->live.erase(it);
  if (latency_s) *latency_s = r->t_done - r->t_arrival;
  if (queue_s) *queue_s = r->t_admit - r->t_arrival;
  if (r->status != EXO_OK) return set_err(r->status, "%s", r->msg.c_str());
  return EXO_OK;
}

extern "C" int exo_server_stats(exo_server* s, exo_server_counters* o) {
  if (!s || !o) return set_err(EXO_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  o->submitted = s->submitted;
  o->admitted = s->admitted;
  o->completed = s->completed;
  o->failed = s->failed;
  o->rejected = s->rejected;
  o->queued = (int64_t)s->queue.size();
  o->in_flight = s->in_flight;
  o->peak_in_flight = s->peak_in_flight;
  o->bypasses = s->bypasses;
  o->mem_budget_bytes = (double)s->cap;
  o->mem_in_use_bytes = (double)s->in_use;
  o->mem_peak_bytes = (double)s->peak;
  return EXO_OK;
}
