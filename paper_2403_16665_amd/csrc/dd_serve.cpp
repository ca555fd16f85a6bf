// dd_serve.cpp -- request server: continuous batching of alpha-dense DFTs
// (each request the problem of Section 2 for one signal) on one device.
//
// Submitters queue requests under a mutex; one scheduler thread owns the
// device side.  Its loop: retire the slots whose completion event has fired
// (stamping their requests done and returning their footprint and scratch),
// then, if a slot is free, admit queued requests in arrival order while the
// batch size, the footprint budget and the scratch pool allow, fill the
// slot's pinned descriptor table and replay the slot's captured graph of the
// persistent batch launch (dd_batch.hip).  Requests outside the batch kernel
// (FP64 dtypes, lengths it is not built for) and every request of the plain
// mode run as plain executions from a resident plan cache, with workspaces
// carved from the same pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/dense_dft.h"
#include "dd_batch_host.hpp"
#include "dd_launch.hpp"
#include "dd_admit.hpp"
#include "dd_pool.hpp"

using namespace dd;

namespace {


uint64_t clock_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  uint64_t ticket = 0;
  dd_desc d{};
  bool kernel = false;  // runs in the persistent batch kernel
  Sched sc;
  size_t footprint = 0;  // input + output + scratch bytes
  size_t scratch = 0;    // bytes taken from the pool while it runs
  size_t scratch_off = 0;
  bool done = false;
  dd_result res{};
};

// Grid variants of a slot's captured batch launch: variant v runs at most
// 16 * 4^v blocks per queue kernel (the last: the device's occupancy), and a
// batch replays the smallest variant whose grids cover its task counts, so a
// batch of a few requests does not pay a device-wide launch.
constexpr int GRID_VARIANTS = 4;
inline int variant_grid(int v, int full) {
  return v == GRID_VARIANTS - 1 ? full : std::min(full, 16 << (2 * v));
}


struct Slot {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t done = nullptr;
  // graphs of the batch launch per grid variant: [0] one queue launch (no
  // two-pass item), [1] both; their staging kernel reads `tab` at every replay
  hipGraph_t graph[2][GRID_VARIANTS] = {};
  hipGraphExec_t exec[2][GRID_VARIANTS] = {};
  BatchTable tab;
  std::vector<Req*> reqs;
  bool busy = false;
};

using PlanKey = std::tuple<int64_t, int, uint64_t, int>;  // N, alpha, bits of T, dtype

}  // namespace

struct dd_server {
  dd_server_cfg cfg{};
  int grid1 = 1, grid2 = 1;
  std::thread worker;
  std::mutex mu;  // queue, tickets, budget, pool ranges, slots' request lists, stats
  std::condition_variable cv_work, cv_done;
  // bumped (under mu) with every notification of cv_work, so that the
  // scheduler can poll for work without the lock
  std::atomic<uint64_t> wake_gen{0};
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  size_t used = 0;
  unsigned char* pool = nullptr;
  RangeAlloc ranges;
  std::mutex mu_res;  // resident tables and plans
  std::map<std::pair<int64_t, int>, ClassTables> classes;
  std::map<PlanKey, dd_plan_t> plans;
  hipStream_t setup = nullptr;
  std::vector<Slot> slots;
  bool stop = false, paused = false;
  dd_server_stats stats{};
};

namespace {

bool plain_mode(const dd_server* s) { return s->cfg.mode == DD_SERVE_PLAIN; }

// Tables of the request's class, generated once on the setup stream.
dd_status class_tables(dd_server* s, const dd_desc& d, const Sched& sc, const ClassTables** out) {
  const auto key = std::make_pair(d.N, (int)d.alpha);
  auto it = s->classes.find(key);
  if (it == s->classes.end()) {
    ClassTables ct;
    dd_status st = make_class_tables(d.N, d.alpha, sc, (s->cfg.flags & DD_TWIDDLE_FP32) != 0, s->setup, &ct);
    if (st == DD_OK) st = hip_status(hipStreamSynchronize(s->setup));
    if (st != DD_OK) {
      free_class_tables(ct);
      return st;
    }
    it = s->classes.emplace(key, ct).first;
  }
  *out = &it->second;
  return DD_OK;
}

dd_status plain_plan(dd_server* s, const dd_desc& d, dd_plan_t* out) {
  uint64_t tb;
  std::memcpy(&tb, &d.T, sizeof(tb));
  const PlanKey key{d.N, (int)d.alpha, tb, (int)d.dtype};
  auto it = s->plans.find(key);
  if (it == s->plans.end()) {
    dd_plan_t p = nullptr;
    const dd_status st = dense_dft_plan(&p, d.N, d.alpha, d.T, 1, d.dtype, (s->cfg.flags & DD_TWIDDLE_FP32) | DD_NO_WORKSPACE);
    if (st != DD_OK) return st;
    it = s->plans.emplace(key, p).first;
  }
  *out = it->second;
  return DD_OK;
}

// Retire a request (called with mu held).
void finish(dd_server* s, Req* r, dd_status st, uint64_t t) {
  r->res.status = st;
  r->res.t_done_ns = t;
  r->done = true;
  s->used -= r->footprint;
  if (r->scratch) s->ranges.release(r->scratch_off, r->scratch);
  s->stats.completed++;
}

// Admit queued requests into `slot` and launch them (called with mu held
// through `lk`; releases it around the device calls).  False if nothing was
// admitted.
bool launch_slot(dd_server* s, Slot& slot, std::unique_lock<std::mutex>& lk) {
  const int cap = plain_mode(s) ? 1 : s->cfg.max_batch;
  std::vector<Req*> take;
  // claims a request's share of the budget and its scratch from the pool
  auto reserve = [&](Req* r) {
    if (s->used + r->footprint > s->cfg.hbm_budget_bytes) return false;
    size_t off = 0;
    if (r->scratch && !s->ranges.alloc(r->scratch, &off)) return false;
    r->scratch_off = off;
    s->used += r->footprint;
    s->stats.peak_footprint = std::max(s->stats.peak_footprint, s->used);
    return true;
  };
  // light load: as long as every queued request can have a free slot of its
  // own, the head goes alone (requests then run concurrently, each at its
  // solo latency; a batch only pays once requests outnumber the free
  // slots); deterministic mode batches whatever is queued (results must not
  // depend on the mix, so a request never takes the plain path instead)
  int free_slots = 0;
  for (const Slot& o : s->slots) free_slots += o.busy ? 0 : 1;
  const int solo_upto = (s->cfg.flags & DD_SERVE_DETERMINISTIC) ? 0 : free_slots;
  admit_requests(s->pending, cap, plain_mode(s), [](const Req* r) { return r->kernel; }, reserve, take,
                 solo_upto);
  if (take.empty()) return false;
  slot.busy = true;
  lk.unlock();

  // a batch of one runs as a plain execution unless results must not
  // depend on the mix
  const bool solo_plain = take.size() == 1 && !(s->cfg.flags & DD_SERVE_DETERMINISTIC);
  std::vector<Req*> kreq, freq;
  for (Req* r : take) (r->kernel && !solo_plain ? kreq : freq).push_back(r);
  std::stable_sort(kreq.begin(), kreq.end(), [](const Req* a, const Req* b) {
    return (int64_t)a->d.alpha * a->d.N > (int64_t)b->d.alpha * b->d.N;
  });
  dd_status st = DD_OK;
  {
    std::lock_guard<std::mutex> rg(s->mu_res);
    for (size_t i = 0; i < kreq.size() && st == DD_OK; ++i) {
      const Req* r = kreq[i];
      const ClassTables* ct = nullptr;
      st = class_tables(s, r->d, r->sc, &ct);
      if (st == DD_OK) {
        // the schedule is the class's, fixed when its tables were made (the
        // tuning table may have changed since the request was classified);
        // every request reserves one spectrum of scratch, enough for either
        cx<float>* Y = ct->sc.single ? nullptr : reinterpret_cast<cx<float>*>(s->pool + r->scratch_off);
        fill_item(slot.tab.items()[i], r->d, *ct, Y);
      }
    }
    // (plain-mode slots have no descriptor table: kreq is empty there)
    if (st == DD_OK && !kreq.empty()) assign_task_offsets(slot.tab.items(), (int)kreq.size(), slot.tab.host);
    const uint64_t t0 = clock_ns();
    for (Req* r : take) r->res.t_start_ns = t0;
    if (st == DD_OK && !kreq.empty()) {
      const BatchMeta& m = *slot.tab.host;
      int v = 0;
      while (v < GRID_VARIANTS - 1 &&
             (variant_grid(v, s->grid1) < std::min(m.n_first, s->grid1) ||
              variant_grid(v, s->grid2) < std::min(m.n_second, s->grid2)))
        ++v;
      st = hip_status(hipGraphLaunch(slot.exec[m.n_second > 0 ? 1 : 0][v], slot.stream));
    }
    for (size_t i = 0; i < freq.size() && st == DD_OK; ++i) {
      Req* r = freq[i];
      dd_plan_t p = nullptr;
      st = plain_plan(s, r->d, &p);
      if (st == DD_OK) st = dense_dft_exec(p, r->d.x, r->d.X, r->scratch ? s->pool + r->scratch_off : nullptr, slot.stream);
    }
    if (st == DD_OK) st = hip_status(hipEventRecord(slot.done, slot.stream));
  }

  lk.lock();
  for (Req* r : take) r->res.batch_requests = (int32_t)take.size();
  s->stats.batches++;
  s->stats.kernel_requests += kreq.size();
  s->stats.fallback_requests += freq.size();
  s->stats.max_batch_seen = std::max(s->stats.max_batch_seen, (int32_t)take.size());
  if (st != DD_OK) {
    // nothing of this batch can be relied on: wait for what was enqueued,
    // then fail its requests
    lk.unlock();
    (void)hipStreamSynchronize(slot.stream);
    lk.lock();
    const uint64_t t = clock_ns();
    for (Req* r : take) finish(s, r, st, t);
    slot.busy = false;
    s->cv_done.notify_all();
    return true;
  }
  slot.reqs = std::move(take);
  return true;
}

void worker_main(dd_server* s) {
  (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progressed = false, any_busy = false;
    for (Slot& sl : s->slots) {
      if (!sl.busy || sl.reqs.empty()) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      const uint64_t t = clock_ns();
      const dd_status st = q == hipSuccess ? DD_OK : DD_ERR_DEVICE;
      for (Req* r : sl.reqs) finish(s, r, st, t);
      sl.reqs.clear();
      sl.busy = false;
      progressed = true;
    }
    if (progressed) s->cv_done.notify_all();
    if (!s->paused && !s->pending.empty()) {
      for (Slot& sl : s->slots) {
        if (sl.busy) continue;
        if (launch_slot(s, sl, lk)) {
          progressed = true;
          any_busy = any_busy || sl.busy;
        }
        break;
      }
    }
    if (s->stop && s->pending.empty() && !any_busy) {
      bool idle = true;
      for (const Slot& sl : s->slots) idle = idle && !sl.busy;
      if (idle) break;
    }
    if (progressed) continue;
    if (any_busy) {
      // work on the device: poll its events again soon
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else if (s->cfg.spin_us > 0 && !s->paused && !s->stop) {
      // idle: poll for a new request for spin_us, then sleep
      const uint64_t seen = s->wake_gen.load(std::memory_order_relaxed);
      lk.unlock();
      const uint64_t until = clock_ns() + (uint64_t)s->cfg.spin_us * 1000u;
      while (s->wake_gen.load(std::memory_order_acquire) == seen && clock_ns() < until) {
      }
      lk.lock();
      if (s->wake_gen.load(std::memory_order_relaxed) == seen) s->cv_work.wait(lk);
    } else {
      s->cv_work.wait(lk);
    }
  }
}

void free_slot(Slot& sl) {
  for (int g = 0; g < 2; ++g)
    for (int v = 0; v < GRID_VARIANTS; ++v) {
      if (sl.exec[g][v]) (void)hipGraphExecDestroy(sl.exec[g][v]);
      if (sl.graph[g][v]) (void)hipGraphDestroy(sl.graph[g][v]);
    }
  if (sl.done) (void)hipEventDestroy(sl.done);
  if (sl.own_stream && sl.stream) (void)hipStreamDestroy(sl.stream);
  free_table(sl.tab);
  sl = Slot{};
}

void free_server(dd_server* s) {
  for (Slot& sl : s->slots) free_slot(sl);
  s->slots.clear();
  for (auto& kv : s->classes) free_class_tables(kv.second);
  s->classes.clear();
  for (auto& kv : s->plans) dense_dft_destroy(kv.second);
  s->plans.clear();
  if (s->pool) (void)hipFree(s->pool);
  s->pool = nullptr;
  if (s->setup) (void)hipStreamDestroy(s->setup);
  s->setup = nullptr;
  for (auto& kv : s->reqs) delete kv.second;
  s->reqs.clear();
}

// One slot: buffers, event, stream, and the graphs of a batch launch over
// its descriptor table (one per grid variant, the largest at the device's
// occupancy at the batch kernel's largest LDS, so that every composition
// has a graph that fits it).
dd_status make_slot(dd_server* s, Slot& sl) {
  const int cap = s->cfg.max_batch;
  dd_status st = DD_OK;
  if (s->cfg.hip_stream) {
    sl.stream = static_cast<hipStream_t>(s->cfg.hip_stream);
  } else {
    st = hip_status(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    sl.own_stream = st == DD_OK;
  }
  if (st == DD_OK) st = hip_status(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  if (plain_mode(s) || st != DD_OK) return st;
  st = alloc_table(sl.tab, cap);
  if (st != DD_OK) return st;
  // a private stream for the captures: the shared caller stream may be in use
  hipStream_t cs = nullptr;
  st = hip_status(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  if (st != DD_OK) return st;
  hipError_t e = hipSuccess;
  for (int g = 0; g < 2 && e == hipSuccess; ++g)
    for (int v = 0; v < GRID_VARIANTS && e == hipSuccess; ++v) {
      e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) break;
      const hipError_t e1 = launch_batch(sl.tab.host_dev, sl.tab.dev, cap, sl.tab.ctl, variant_grid(v, s->grid1),
                                         g ? variant_grid(v, s->grid2) : 0, BATCH_LDS_MAX, batch_lds2_max(), cs);
      e = hipStreamEndCapture(cs, &sl.graph[g][v]);
      if (e == hipSuccess) e = e1;
      if (e == hipSuccess) e = hipGraphInstantiate(&sl.exec[g][v], sl.graph[g][v], nullptr, nullptr, 0);
    }
  (void)hipStreamDestroy(cs);
  return hip_status(e);
}

// Schedule, footprint and scratch of a request of this shape (host only).
dd_status classify_shape(const dd_server* s, int64_t N, int alpha, double T, dd_dtype dtype, Req* r) {
  const dd_status st = batch_check_shape(N, alpha, T, dtype);
  if (st != DD_OK) return st;
  r->d.N = N;
  r->d.alpha = alpha;
  r->d.T = T;
  r->d.dtype = dtype;
  const size_t M = (size_t)alpha * N;
  r->kernel = !plain_mode(s) && (dtype == DD_F32 || dtype == DD_C64) &&
              (s->cfg.batch_max_bins < 0 || (int64_t)M <= s->cfg.batch_max_bins) && batch_schedule(N, alpha, &r->sc);
  // scratch for a two-pass kernel item (one spectrum in the request's
  // precision) or a plain execution, which a kernel request alone in its
  // batch may become (its rows may be padded: at most 1/8 more)
  r->scratch = scratch_bytes_bound(M * batch_out_elem(dtype));
  r->footprint = (size_t)N * batch_in_elem(dtype) + M * batch_out_elem(dtype) + round_up(r->scratch, POOL_ALIGN);
  return DD_OK;
}

}  // namespace

extern "C" {

uint64_t dense_dft_clock_ns(void) { return clock_ns(); }

dd_status dense_dft_server_create(const dd_server_cfg* cfg, dd_server_t* out) {
  if (!out) return DD_ERR_INVALID;
  *out = nullptr;
  if (!cfg) return DD_ERR_INVALID;
  dd_server_cfg c = *cfg;
  if (c.mode != DD_SERVE_BATCHED && c.mode != DD_SERVE_PLAIN) return DD_ERR_INVALID;
  if (c.max_inflight < 0 || c.max_inflight > 64 || c.max_batch < 0 || c.max_batch > 4096 || c.max_queue < 0)
    return DD_ERR_INVALID;
  if (c.flags & ~(uint32_t)(DD_TWIDDLE_FP32 | DD_SERVE_DETERMINISTIC)) return DD_ERR_INVALID;
  if (c.batch_max_bins < -1) return DD_ERR_INVALID;
  if (c.spin_us < -1 || c.spin_us > 1000000) return DD_ERR_INVALID;
  if (c.spin_us == 0) c.spin_us = 1000;
  if (c.hbm_budget_bytes == 0) c.hbm_budget_bytes = (size_t)8 << 30;
  if (c.max_inflight == 0) c.max_inflight = 8;
  if (c.max_batch == 0) c.max_batch = 256;
  if (c.mode == DD_SERVE_PLAIN) c.max_batch = 1;
  if (c.max_queue == 0) c.max_queue = 65536;
  if (c.batch_max_bins == 0) c.batch_max_bins = (int64_t)1 << 20;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || c.device < 0 || c.device >= ndev) return DD_ERR_DEVICE;

  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(c.device) != hipSuccess) return DD_ERR_DEVICE;
  dd_server* s = new (std::nothrow) dd_server;
  if (!s) {
    (void)hipSetDevice(prev);
    return DD_ERR_NOMEM;
  }
  s->cfg = c;
  s->stats.pool_bytes = c.hbm_budget_bytes;
  dd_status st = hip_status(hipMalloc((void**)&s->pool, c.hbm_budget_bytes));
  if (st == DD_ERR_DEVICE) st = DD_ERR_NOMEM;
  s->ranges.reset(c.hbm_budget_bytes);
  if (st == DD_OK) st = hip_status(hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking));
  if (st == DD_OK && c.mode == DD_SERVE_BATCHED) st = hip_status(batch_set_lds(BATCH_LDS_MAX, batch_lds2_max()));
  if (st == DD_OK) {
    hipDeviceProp_t prop;
    st = hip_status(hipGetDeviceProperties(&prop, c.device));
    if (st == DD_OK) {
      s->grid1 = prop.multiProcessorCount * batch_max_blocks_per_cu(0, BATCH_LDS_MAX);
      s->grid2 = prop.multiProcessorCount * batch_max_blocks_per_cu(1, batch_lds2_max());
    }
  }
  s->slots.resize(c.max_inflight);
  for (int i = 0; i < c.max_inflight && st == DD_OK; ++i) st = make_slot(s, s->slots[i]);
  if (st == DD_OK) st = hip_status(hipDeviceSynchronize());
  if (st == DD_OK) {
    try {
      s->worker = std::thread(worker_main, s);
    } catch (...) {
      st = DD_ERR_NOMEM;
    }
  }
  if (st != DD_OK) {
    free_server(s);
    delete s;
    (void)hipSetDevice(prev);
    return st;
  }
  (void)hipSetDevice(prev);
  *out = s;
  return DD_OK;
}

dd_status dense_dft_server_warm(dd_server_t s, int64_t N, int32_t alpha, double T, dd_dtype dtype) {
  if (!s) return DD_ERR_INVALID;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return DD_ERR_CLOSED;
  }
  Req r;
  dd_status st = classify_shape(s, N, alpha, T, dtype, &r);
  if (st != DD_OK) return st;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->cfg.device);
  {
    std::lock_guard<std::mutex> rg(s->mu_res);
    // both paths may serve the class: batch-kernel tables and a plain plan
    if (r.kernel) {
      const ClassTables* ct = nullptr;
      st = class_tables(s, r.d, r.sc, &ct);
    }
    if (st == DD_OK && (!r.kernel || !(s->cfg.flags & DD_SERVE_DETERMINISTIC))) {
      dd_plan_t p = nullptr;
      st = plain_plan(s, r.d, &p);
    }
  }
  (void)hipSetDevice(prev);
  return st;
}

dd_status dense_dft_submit_at(dd_server_t s, const dd_desc* req, uint64_t t_arrival_ns, uint64_t* ticket) {
  if (!s || !req || !ticket) return DD_ERR_INVALID;
  Req* r = new (std::nothrow) Req;
  if (!r) return DD_ERR_NOMEM;
  dd_status st = batch_check_desc(*req);
  if (st == DD_OK) st = classify_shape(s, req->N, req->alpha, req->T, req->dtype, r);
  if (st == DD_OK) r->d = *req;
  if (st == DD_OK && r->footprint > s->cfg.hbm_budget_bytes) st = DD_ERR_TOO_LARGE;
  if (st != DD_OK) {
    delete r;
    return st;
  }
  r->res.t_arrival_ns = t_arrival_ns;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) st = DD_ERR_CLOSED;
    else if ((int64_t)s->pending.size() >= s->cfg.max_queue) st = DD_ERR_BUSY;
    if (st != DD_OK) {
      delete r;
      return st;
    }
    r->ticket = s->next_ticket++;
    s->pending.push_back(r);
    s->wake_gen.fetch_add(1, std::memory_order_release);
    s->reqs.emplace(r->ticket, r);
    s->stats.submitted++;
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return DD_OK;
}

dd_status dense_dft_submit(dd_server_t s, const dd_desc* req, uint64_t* ticket) {
  return dense_dft_submit_at(s, req, clock_ns(), ticket);
}

dd_status dense_dft_submit_many_at(dd_server_t s, const dd_desc* reqs, const uint64_t* t_arrival_ns, int32_t count,
                                   uint64_t* tickets, int32_t* submitted) {
  if (!submitted) return DD_ERR_INVALID;
  *submitted = 0;
  if (!s || count < 0 || (count > 0 && (!reqs || !t_arrival_ns || !tickets))) return DD_ERR_INVALID;
  for (int32_t i = 0; i < count; ++i) {
    if (i > 0 && t_arrival_ns[i] < t_arrival_ns[i - 1]) return DD_ERR_INVALID;
    while (clock_ns() < t_arrival_ns[i]) {
    }
    const dd_status st = dense_dft_submit_at(s, &reqs[i], t_arrival_ns[i], &tickets[i]);
    if (st != DD_OK) return st;
    *submitted = i + 1;
  }
  return DD_OK;
}

dd_status dense_dft_poll(dd_server_t s, uint64_t ticket, dd_result* r) {
  if (!s || !r) return DD_ERR_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return DD_ERR_INVALID;
  if (!it->second->done) return DD_ERR_BUSY;
  *r = it->second->res;
  delete it->second;
  s->reqs.erase(it);
  return DD_OK;
}

dd_status dense_dft_wait(dd_server_t s, uint64_t ticket, int64_t timeout_us, dd_result* r) {
  if (!s || !r) return DD_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second->done;
  };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return DD_ERR_TIMEOUT;
  }
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return DD_ERR_INVALID;
  *r = it->second->res;
  delete it->second;
  s->reqs.erase(it);
  return DD_OK;
}

dd_status dense_dft_server_pause(dd_server_t s, int32_t paused) {
  if (!s) return DD_ERR_INVALID;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->paused = paused != 0;
    s->wake_gen.fetch_add(1, std::memory_order_release);
  }
  s->cv_work.notify_one();
  return DD_OK;
}

dd_status dense_dft_server_stats(dd_server_t s, dd_server_stats* st) {
  if (!s || !st) return DD_ERR_INVALID;
  std::lock_guard<std::mutex> g(s->mu);
  *st = s->stats;
  {
    std::lock_guard<std::mutex> rg(s->mu_res);
    st->classes = (int32_t)s->classes.size();
  }
  return DD_OK;
}

dd_status dense_dft_server_destroy(dd_server_t s) {
  if (!s) return DD_ERR_INVALID;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->paused = false;
    s->wake_gen.fetch_add(1, std::memory_order_release);
  }
  s->cv_work.notify_one();
  if (s->worker.joinable()) s->worker.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->cfg.device);
  (void)hipDeviceSynchronize();
  free_server(s);
  (void)hipSetDevice(prev);
  s->cv_done.notify_all();
  delete s;
  return DD_OK;
}

}  // extern "C"
