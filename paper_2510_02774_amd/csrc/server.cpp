// server.cpp -- continuous batching of graph builds on one GPU.
//
// A host thread admits queued requests in arrival order whenever a slot
// (stream) is free and the caller's arena has room for the build's
// workspace, enqueues the whole build on the slot's stream, and retires it
// once its completion event has passed, freeing the slot and the arena range
// for the next request. Builds in different slots overlap on the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "grnnd.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr size_t kArenaAlign = 256;

struct Record {
  grnnd_request req;
  grnnd_params params;
  size_t bytes = 0;
  int32_t state = GRNND_REQ_QUEUED;
  Clock::time_point submitted;
  double latency = 0.0;
};

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t next = it->first + bytes;
        free_.erase(it);
        if (rest) free_[next] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;  // the requests of the build it runs
  size_t off = 0, bytes = 0;
};

// Requests that can share one batched build: equal d, metric, R and
// parameters.
bool same_class(const Record& a, const Record& b) {
  return a.req.d == b.req.d && a.req.metric == b.req.metric && a.req.R == b.req.R &&
         std::memcmp(&a.params, &b.params, sizeof(grnnd_params)) == 0;
}

}  // namespace

namespace grnnd {
int set_error(int code, const char* msg);  // api.cpp: the thread's last-error text
}

namespace {
int sfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return grnnd::set_error(code, buf);
}
}  // namespace

struct grnnd_server {
  char* arena = nullptr;
  size_t budget = 0;
  int device = 0;
  Arena alloc{0};
  std::vector<Slot> slots;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Record> recs;
  uint64_t next_ticket = 1;
  grnnd_server_stats stats{};
  std::mutex mu;
  std::condition_variable cv;  // wakes the admission thread
  std::condition_variable idle;  // signals completions to drain()
  bool stop = false;
  std::thread worker;
  // batching: queued requests of one class, each of at most batch_points
  // points, share one build (grnnd_build_batch) of at most batch_max
  // requests and batch_points points in all
  int32_t batch_max = 16;
  int64_t batch_points = 1 << 18;

  int inflight() const {
    int k = 0;
    for (const Slot& sl : slots) k += sl.busy;
    return k;
  }

  // Admission and retirement loop (the only thread that launches work).
  void run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      // retire finished builds
      bool retired = false;
      for (Slot& sl : slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        for (uint64_t tk : sl.tickets) {
          Record& r = recs[tk];
          r.latency = std::chrono::duration<double>(Clock::now() - r.submitted).count();
          if (q == hipSuccess) {
            r.state = GRNND_REQ_DONE;
            ++stats.completed;
          } else {
            r.state = GRNND_EDEVICE;
            ++stats.failed;
          }
        }
        alloc.release(sl.off, sl.bytes);
        sl.busy = false;
        retired = true;
      }
      if (retired) idle.notify_all();
      // admit in arrival order while a slot and arena room are free
      while (!pending.empty()) {
        Slot* free_slot = nullptr;
        for (Slot& sl : slots)
          if (!sl.busy) {
            free_slot = &sl;
            break;
          }
        if (!free_slot) break;
        const uint64_t t = pending.front();
        Record& r = recs[t];
        // the head request, with the queued requests of its class that fit
        // the batch limits (a batch of one is a plain build)
        std::vector<uint64_t> batch{t};
        std::vector<int64_t> ns{r.req.n};
        int64_t pts = r.req.n;
        if (batch_max > 1 && r.req.n <= batch_points) {
          for (size_t k = 1; k < pending.size() && (int32_t)batch.size() < batch_max; ++k) {
            const Record& o = recs[pending[k]];
            if (!same_class(r, o) || o.req.n > batch_points || pts + o.req.n > batch_points)
              continue;
            batch.push_back(pending[k]);
            ns.push_back(o.req.n);
            pts += o.req.n;
          }
        }
        size_t bytes = r.bytes, off = 0;
        while (batch.size() > 1) {
          if (grnnd_batch_workspace_size(ns.data(), (int32_t)ns.size(), r.req.d, r.req.R,
                                         &r.params, &bytes) == GRNND_OK &&
              alloc.alloc(bytes, &off))
            break;
          batch.pop_back();  // too large for the room left: a smaller batch
          ns.pop_back();
        }
        if (batch.size() == 1) {
          bytes = r.bytes;
          if (!alloc.alloc(bytes, &off)) break;  // wait for room (head of the line keeps its turn)
        }
        for (uint64_t tk : batch) {
          pending.erase(std::find(pending.begin(), pending.end(), tk));
          recs[tk].state = GRNND_REQ_RUNNING;
        }
        free_slot->busy = true;
        free_slot->tickets = batch;
        free_slot->off = off;
        free_slot->bytes = bytes;
        if (batch.size() > 1) {
          ++stats.batches;
          stats.batched_requests += (int64_t)batch.size();
        }
        const uint64_t used = alloc.used();
        if (used > stats.peak_arena_bytes) stats.peak_arena_bytes = used;
        const int64_t nin = inflight();
        if (nin > stats.peak_inflight) stats.peak_inflight = nin;
        const grnnd_params p = r.params;
        std::vector<grnnd_batch_item> items;
        for (uint64_t tk : batch) {
          const grnnd_request& q = recs[tk].req;
          items.push_back(grnnd_batch_item{q.points, q.n, q.seed, q.out_adj, q.out_keys});
        }
        const grnnd_request q = r.req;
        Slot* sl = free_slot;
        lk.unlock();
        int rc = batch.size() == 1
                     ? grnnd_build_ex(q.points, q.n, q.d, q.metric, q.R, &p, q.seed, q.out_adj,
                                      q.out_keys, nullptr, arena + off, bytes, sl->stream)
                     : grnnd_build_batch(items.data(), (int32_t)items.size(), q.d, q.metric, q.R,
                                         &p, nullptr, arena + off, bytes, sl->stream);
        if (rc == GRNND_OK && hipEventRecord(sl->done, sl->stream) != hipSuccess)
          rc = GRNND_EDEVICE;
        // a build that failed part way may have queued kernels on the slot's
        // stream: they finish before its arena range can be handed out again
        if (rc != GRNND_OK) (void)hipStreamSynchronize(sl->stream);
        lk.lock();
        if (rc != GRNND_OK) {
          for (uint64_t tk : batch) {
            Record& rr = recs[tk];
            rr.state = rc;
            rr.latency = std::chrono::duration<double>(Clock::now() - rr.submitted).count();
            ++stats.failed;
          }
          alloc.release(off, bytes);
          sl->busy = false;
          idle.notify_all();
        }
      }
      if (stop && pending.empty() && inflight() == 0) break;
      // sleep until a submission, or poll the running builds shortly
      if (inflight() > 0)
        cv.wait_for(lk, std::chrono::microseconds(50));
      else
        cv.wait(lk, [&] { return stop || !pending.empty(); });
    }
  }
};

extern "C" {

int grnnd_server_create(void* arena, size_t budget_bytes, int32_t slots, grnnd_server** out) {
  if (!out) return sfail(GRNND_EINVAL, "out is null");
  *out = nullptr;
  if (!arena || budget_bytes == 0) return sfail(GRNND_EINVAL, "arena is null or empty");
  if (reinterpret_cast<uintptr_t>(arena) & (kArenaAlign - 1))
    return sfail(GRNND_EINVAL, "arena must be 256-byte aligned");
  if (slots < 1 || slots > 64) return sfail(GRNND_EINVAL, "slots=%d out of range [1, 64]", slots);
  auto* s = new grnnd_server();
  s->arena = static_cast<char*>(arena);
  s->budget = budget_bytes;
  s->alloc = Arena(budget_bytes);
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return sfail(GRNND_EDEVICE, "no current device");
  }
  s->slots.resize((size_t)slots);
  for (Slot& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      for (Slot& t : s->slots) {
        if (t.done) (void)hipEventDestroy(t.done);
        if (t.stream) (void)hipStreamDestroy(t.stream);
      }
      delete s;
      return sfail(GRNND_EDEVICE, "cannot create a stream or event");
    }
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return GRNND_OK;
}

int grnnd_server_submit(grnnd_server* s, const grnnd_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return sfail(GRNND_EINVAL, "null argument");
  if (!r->points || !r->out_adj) return sfail(GRNND_EINVAL, "points or out_adj is null");
  if (r->metric != GRNND_METRIC_L2 && r->metric != GRNND_METRIC_IP)
    return sfail(GRNND_EINVAL, "metric=%d unknown", r->metric);
  grnnd_params p;
  if (r->params) {
    p = *r->params;
  } else if (grnnd_params_default(&p, r->R, 4) != GRNND_OK) {
    return sfail(GRNND_EINVAL, "%s", grnnd_last_error());
  }
  size_t bytes = 0;
  if (grnnd_workspace_size(r->n, r->d, r->R, &p, &bytes) != GRNND_OK)
    return sfail(GRNND_EINVAL, "%s", grnnd_last_error());
  if (bytes > s->budget)
    return sfail(GRNND_EBUDGET, "request needs %zu B of workspace, budget is %zu B", bytes,
                 s->budget);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const uint64_t t = s->next_ticket++;
    Record& rec = s->recs[t];
    rec.req = *r;
    rec.params = p;
    rec.req.params = nullptr;
    rec.bytes = bytes;
    rec.submitted = Clock::now();
    s->pending.push_back(t);
    ++s->stats.submitted;
    *ticket = t;
  }
  s->cv.notify_all();
  return GRNND_OK;
}

int grnnd_server_poll(grnnd_server* s, uint64_t ticket, int32_t* state, double* latency_s) {
  if (!s) return sfail(GRNND_EINVAL, "server is null");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->recs.find(ticket);
  if (it == s->recs.end()) return sfail(GRNND_EINVAL, "unknown ticket %llu",
                                        (unsigned long long)ticket);
  if (state) *state = it->second.state;
  if (latency_s) *latency_s = it->second.latency;
  return GRNND_OK;
}

int grnnd_server_drain(grnnd_server* s) {
  if (!s) return sfail(GRNND_EINVAL, "server is null");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.notify_all();
  s->idle.wait(lk, [&] { return s->pending.empty() && s->inflight() == 0; });
  return GRNND_OK;
}

int grnnd_server_set_batch(grnnd_server* s, int32_t max_requests, int64_t max_points) {
  if (!s) return sfail(GRNND_EINVAL, "server is null");
  if (max_requests < 1 || max_requests > 64)
    return sfail(GRNND_EINVAL, "max_requests=%d out of range [1, 64]", max_requests);
  if (max_points < 2) return sfail(GRNND_EINVAL, "max_points must be >= 2");
  std::lock_guard<std::mutex> lk(s->mu);
  s->batch_max = max_requests;
  s->batch_points = max_points;
  return GRNND_OK;
}

int grnnd_server_stats_read(grnnd_server* s, grnnd_server_stats* out) {
  if (!s || !out) return sfail(GRNND_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return GRNND_OK;
}

int grnnd_server_destroy(grnnd_server* s) {
  if (!s) return sfail(GRNND_EINVAL, "server is null");
  grnnd_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (Slot& sl : s->slots) {
    (void)hipEventDestroy(sl.done);
    (void)hipStreamDestroy(sl.stream);
  }
  delete s;
  return GRNND_OK;
}

}  // extern "C"
