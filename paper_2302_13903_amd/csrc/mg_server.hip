// mg_server.hip -- serving runtime: many independent solves on one device (see include/mg355.h).
//
// Host code only.  The calling thread of mg_server_run is the dispatcher: it submits each
// request at its arrival time into a pending queue.  `workers` threads, one HIP stream each,
// take requests from the queue when their hierarchy fits the HBM budget, run mg_solve on
// their stream and release the hierarchy, which stays resident for the next request of the
// same workspace class (n, precision, MeshBlock side, scheme).  All bookkeeping (queue, pool, counters) is under one mutex; device
// allocation, release and the solves themselves run outside it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mg355.h"

namespace {

using Clock = std::chrono::steady_clock;

// Workspace class of a request: solves of one class need the same workspace (size,
// precision, MeshBlock side for the block layout, scheme), so one resident hierarchy serves
// every request of its class.
struct Class {
  int n = 0, precision = 0, block_n = 0, scheme = 0;
  bool operator==(const Class& o) const {
    return n == o.n && precision == o.precision && block_n == o.block_n && scheme == o.scheme;
  }
};

Class class_of(const mg_params& p) {
  return Class{p.n, p.precision, p.layout == MG_LAYOUT_BLOCKS ? p.block_n : 0, p.scheme};
}

// A resident hierarchy: one solver context sized for its class (with that footprint as the
// context's HBM budget, so it never grows beyond what admission counted) plus an n^3 result
// slot.
struct Entry {
  Class cls;
  mg_params params{};        // parameters the context is reserved for
  size_t bytes = 0;
  mg_ctx* ctx = nullptr;
  double* slot = nullptr;
  bool busy = false;
  bool ready = false;        // allocated (a reserved entry is allocated by its first user)
  uint64_t last_used = 0;
};

size_t entry_bytes(const mg_params& p) {
  const size_t fp = mg_footprint_bytes(&p);
  if (fp == 0) return 0;
  return fp + (size_t)p.n * p.n * p.n * sizeof(double) + 256;
}

}  // namespace

struct mg_server {
  mg_server_config cfg{};
  std::string err;
  std::vector<hipStream_t> streams;
  std::mutex m;
  std::condition_variable cv;
  std::vector<std::unique_ptr<Entry>> pool;
  size_t used = 0;
  uint64_t tick = 0;
  mg_server_stats stats{};
  int in_flight = 0;
  // state of the current run
  std::deque<int> pending;
  bool all_submitted = false;
  mg_request* reqs = nullptr;
  Clock::time_point t0;
};

namespace {

double ms_since(const mg_server* s) {
  return std::chrono::duration<double, std::milli>(Clock::now() - s->t0).count();
}

void release_entry_memory(mg_server* s, Entry* e) {
  if (s->cfg.simulate) return;
  if (e->ctx) mg_ctx_destroy(e->ctx);
  if (e->slot) {
    (void)hipSetDevice(s->cfg.device);
    (void)hipFree(e->slot);
  }
  e->ctx = nullptr;
  e->slot = nullptr;
}

// Allocate the context and slot of a reserved entry (outside the lock).
int materialise(mg_server* s, Entry* e) {
  if (s->cfg.simulate) {
    e->ready = true;
    return MG_OK;
  }
  const mg_params& p = e->params;
  int st = mg_ctx_create(&e->ctx, s->cfg.device, mg_footprint_bytes(&p));
  if (st != MG_OK) return st;
  // one stream per worker: the split passes' second stream would share the device's few
  // hardware queues with the other workers' streams (measured slower in the request mix)
  st = mg_tuning_set(e->ctx, "split fp64 0\n");
  if (st != MG_OK) return st;
  st = mg_ctx_reserve(e->ctx, &p);
  if (st != MG_OK) return st;
  if (hipMalloc((void**)&e->slot, (size_t)p.n * p.n * p.n * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return MG_ERR_OOM;
  }
  e->ready = true;
  return MG_OK;
}

// Under the lock: find or make room for an entry of the class of p.  Idle entries of other
// classes that must go to make room are moved into `evict` (the caller frees them unlocked).
// Returns nullptr when the request must wait.
Entry* acquire_locked(mg_server* s, const mg_params& p, size_t bytes, std::vector<std::unique_ptr<Entry>>& evict,
                      bool* reused) {
  const Class cls = class_of(p);
  for (auto& e : s->pool)
    if (!e->busy && e->cls == cls) {
      e->busy = true;
      e->last_used = ++s->tick;
      *reused = e->ready;
      return e.get();
    }
  size_t idle_other = 0;
  for (auto& e : s->pool)
    if (!e->busy) idle_other += e->bytes;
  if (s->used + bytes > s->cfg.hbm_budget && s->used - idle_other + bytes > s->cfg.hbm_budget) return nullptr;
  while (s->used + bytes > s->cfg.hbm_budget) {
    auto victim = s->pool.end();
    for (auto it = s->pool.begin(); it != s->pool.end(); ++it)
      if (!(*it)->busy && (victim == s->pool.end() || (*it)->last_used < (*victim)->last_used)) victim = it;
    if (victim == s->pool.end()) return nullptr;  // cannot happen after the check above
    s->used -= (*victim)->bytes;
    evict.push_back(std::move(*victim));
    s->pool.erase(victim);
    s->stats.evicted++;
  }
  auto e = std::make_unique<Entry>();
  e->cls = cls;
  e->params = p;
  e->bytes = bytes;
  e->busy = true;
  e->last_used = ++s->tick;
  s->used += bytes;
  s->stats.created++;
  s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->used);
  *reused = false;
  s->pool.push_back(std::move(e));
  return s->pool.back().get();
}

// Under the lock: the next request a worker may start, per policy; rejects requests that
// can never fit.  Returns -1 when none can start now.
int pick_locked(mg_server* s, Entry** out, std::vector<std::unique_ptr<Entry>>& evict, bool* reused) {
  for (size_t q = 0; q < s->pending.size();) {
    const int id = s->pending[q];
    mg_request& r = s->reqs[id];
    const size_t bytes = entry_bytes(r.params);
    if (bytes == 0 || bytes > s->cfg.hbm_budget) {
      r.status = bytes == 0 ? MG_ERR_INVALID_ARG : MG_ERR_OOM;
      r.admit_ms = r.start_ms = r.end_ms = ms_since(s);
      r.worker = -1;
      s->stats.rejected++;
      s->pending.erase(s->pending.begin() + q);
      continue;
    }
    Entry* e = acquire_locked(s, r.params, bytes, evict, reused);
    if (e) {
      s->pending.erase(s->pending.begin() + q);
      *out = e;
      return id;
    }
    if (s->cfg.policy == MG_SERVE_FIFO) return -1;
    ++q;
  }
  return -1;
}

void worker_main(mg_server* s, int w) {
  if (!s->cfg.simulate) (void)hipSetDevice(s->cfg.device);
  std::vector<std::unique_ptr<Entry>> evict;
  for (;;) {
    Entry* e = nullptr;
    bool reused = false;
    int id = -1;
    {
      std::unique_lock<std::mutex> lk(s->m);
      s->cv.wait(lk, [&] {
        id = pick_locked(s, &e, evict, &reused);
        return id >= 0 || (s->all_submitted && s->pending.empty());
      });
      if (id < 0) {
        lk.unlock();
        s->cv.notify_all();  // requests rejected while waiting may have emptied the queue
        return;
      }
      s->in_flight++;
      s->stats.max_concurrent = std::max(s->stats.max_concurrent, s->in_flight);
      if (reused) s->stats.reused++;
    }
    for (auto& v : evict) release_entry_memory(s, v.get());
    evict.clear();
    mg_request& r = s->reqs[id];
    r.admit_ms = ms_since(s);
    r.worker = w;
    r.reused = reused ? 1 : 0;
    int st = e->ready ? MG_OK : materialise(s, e);
    r.start_ms = ms_since(s);
    if (st == MG_OK) {
      if (s->cfg.simulate) {
        std::this_thread::sleep_for(std::chrono::duration<double, std::milli>(std::max(0.0, r.sim_ms)));
        r.n_hist = 0;
        r.resid = 0;
      } else if (r.params.mode == MG_MODE_MGI && !r.phi) {
        st = MG_ERR_INVALID_ARG;
      } else {
        const int cap = std::max(r.params.max_cycles, r.params.fixed_cycles) + 1;
        std::vector<double> hist((size_t)cap);
        int nh = 0;
        st = mg_solve(e->ctx, &r.params, &r.bc, r.rho, r.phi ? r.phi : e->slot, hist.data(), &nh, s->streams[w]);
        r.n_hist = nh;
        r.resid = nh > 0 ? hist[(size_t)nh - 1] : 0.0;
        if (r.hist && r.hist_cap > 0)
          for (int i = 0; i < std::min(nh, r.hist_cap); ++i) r.hist[i] = hist[(size_t)i];
      }
    }
    r.status = st;
    r.end_ms = ms_since(s);
    {
      std::lock_guard<std::mutex> lk(s->m);
      s->in_flight--;
      if (!e->ready) {
        // allocation failed: drop the entry and its accounting
        for (auto it = s->pool.begin(); it != s->pool.end(); ++it)
          if (it->get() == e) {
            s->used -= e->bytes;
            evict.push_back(std::move(*it));
            s->pool.erase(it);
            break;
          }
      } else {
        e->busy = false;
        e->last_used = ++s->tick;
      }
    }
    for (auto& v : evict) release_entry_memory(s, v.get());
    evict.clear();
    s->cv.notify_all();
  }
}

}  // namespace

extern "C" {

int mg_server_create(mg_server** out, const mg_server_config* cfg) {
  if (!out || !cfg) return MG_ERR_INVALID_ARG;
  *out = nullptr;
  if (cfg->workers < 1 || cfg->workers > 64) return MG_ERR_INVALID_ARG;
  if (cfg->policy != MG_SERVE_FIFO && cfg->policy != MG_SERVE_SKIP) return MG_ERR_INVALID_ARG;
  auto* s = new mg_server();
  s->cfg = *cfg;
  if (!cfg->simulate) {
    if (hipSetDevice(cfg->device) != hipSuccess) {
      delete s;
      return MG_ERR_DEVICE;
    }
    if (cfg->hbm_budget == 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        delete s;
        return MG_ERR_DEVICE;
      }
      s->cfg.hbm_budget = fr / 10 * 8;
    }
    for (int w = 0; w < cfg->workers; ++w) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        mg_server_destroy(s);
        return MG_ERR_DEVICE;
      }
      s->streams.push_back(st);
    }
  } else if (cfg->hbm_budget == 0) {
    delete s;
    return MG_ERR_INVALID_ARG;  // simulate mode has no device to ask
  }
  *out = s;
  return MG_OK;
}

void mg_server_destroy(mg_server* s) {
  if (!s) return;
  for (auto& e : s->pool) release_entry_memory(s, e.get());
  s->pool.clear();
  if (!s->cfg.simulate) {
    (void)hipSetDevice(s->cfg.device);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
  }
  delete s;
}

const char* mg_server_last_error(const mg_server* s) { return s ? s->err.c_str() : "null server"; }

int mg_server_reserve(mg_server* s, const mg_params* p, int count) {
  if (!s || !p || count < 0) return MG_ERR_INVALID_ARG;
  const size_t bytes = entry_bytes(*p);
  if (bytes == 0) return MG_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    Entry* e = nullptr;
    {
      std::lock_guard<std::mutex> lk(s->m);
      if (s->used + bytes > s->cfg.hbm_budget) {
        s->err = "reserve: budget exhausted";
        return MG_ERR_OOM;
      }
      auto ne = std::make_unique<Entry>();
      ne->cls = class_of(*p);
      ne->params = *p;
      ne->bytes = bytes;
      ne->busy = true;
      ne->last_used = ++s->tick;
      s->used += bytes;
      s->stats.created++;
      s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->used);
      e = ne.get();
      s->pool.push_back(std::move(ne));
    }
    const int st = materialise(s, e);
    std::lock_guard<std::mutex> lk(s->m);
    if (st != MG_OK) {
      for (auto it = s->pool.begin(); it != s->pool.end(); ++it)
        if (it->get() == e) {
          s->used -= e->bytes;
          release_entry_memory(s, e);
          s->pool.erase(it);
          break;
        }
      s->err = "reserve: allocation failed";
      return st;
    }
    e->busy = false;
  }
  return MG_OK;
}

int mg_server_run(mg_server* s, mg_request* reqs, int n) {
  if (!s || (n > 0 && !reqs) || n < 0) return MG_ERR_INVALID_ARG;
  std::vector<int> order((size_t)n);
  for (int i = 0; i < n; ++i) {
    order[(size_t)i] = i;
    reqs[i].status = MG_ERR_INVALID_ARG;
    reqs[i].n_hist = 0;
    reqs[i].resid = 0;
    reqs[i].admit_ms = reqs[i].start_ms = reqs[i].end_ms = 0;
    reqs[i].worker = -1;
    reqs[i].reused = 0;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival_ms < reqs[b].arrival_ms; });
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->pending.clear();
    s->all_submitted = false;
    s->reqs = reqs;
    s->t0 = Clock::now();
  }
  std::vector<std::thread> th;
  for (int w = 0; w < s->cfg.workers; ++w) th.emplace_back(worker_main, s, w);
  for (int id : order) {
    const auto due = s->t0 + std::chrono::duration_cast<Clock::duration>(
                                 std::chrono::duration<double, std::milli>(std::max(0.0, reqs[id].arrival_ms)));
    std::this_thread::sleep_until(due);
    {
      std::lock_guard<std::mutex> lk(s->m);
      s->pending.push_back(id);
    }
    s->cv.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->all_submitted = true;
  }
  s->cv.notify_all();
  for (auto& t : th) t.join();
  s->reqs = nullptr;
  return MG_OK;
}

int mg_server_get_stats(const mg_server* s, mg_server_stats* out) {
  if (!s || !out) return MG_ERR_INVALID_ARG;
  auto* ms = const_cast<mg_server*>(s);
  std::lock_guard<std::mutex> lk(ms->m);
  *out = s->stats;
  out->resident_bytes = s->used;
  return MG_OK;
}

}  // extern "C"
