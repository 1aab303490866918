// Continuous-batching sketch server.
//
// Requests of uneven size arrive from any thread (cabs_submit).  A scheduler
// thread admits them in arrival order as soon as a slot (a HIP stream) is free
// and their workspace fits in the device pool, launches the whole sketch on
// the slot's stream, and retires it when the stream's completion event has
// fired, returning its workspace to the pool.  Requests in different slots run
// concurrently on the device; each one's kernels only touch its own buffers, so
// its result is the same whether it runs alone or next to others.
// The pool is one device allocation made at creation, carved first-fit in
// 256-byte units; nothing is allocated per request.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cabs.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Block { size_t off, size; };

// First-fit allocator over [0, capacity) with coalescing of free neighbours.
class Pool {
 public:
  explicit Pool(size_t cap) { free_.push_back({0, cap}); }
  bool alloc(size_t bytes, size_t& off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].size >= bytes) {
        off = free_[i].off;
        free_[i].off += bytes;
        free_[i].size -= bytes;
        if (free_[i].size == 0) free_.erase(free_.begin() + i);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    size_t i = 0;
    while (i < free_.size() && free_[i].off < off) ++i;
    free_.insert(free_.begin() + i, {off, bytes});
    if (i + 1 < free_.size() && free_[i].off + free_[i].size == free_[i + 1].off) {
      free_[i].size += free_[i + 1].size;
      free_.erase(free_.begin() + i + 1);
    }
    if (i > 0 && free_[i - 1].off + free_[i - 1].size == free_[i].off) {
      free_[i - 1].size += free_[i].size;
      free_.erase(free_.begin() + i);
    }
  }

 private:
  std::vector<Block> free_;
};

enum ReqState { QUEUED, RUNNING, DONE, CANCELED, FAILED };

struct Request {
  uint64_t ticket;
  cabs_matrix mat;
  cabs_params prm;
  cabs_result res;
  int64_t err_samples = 0;
  uint64_t err_seed = 0;
  double* err_out3 = nullptr;
  size_t ws_bytes;
  size_t ws_off = 0;
  int slot = -1;
  ReqState state = QUEUED;
  int status = CABS_OK;
  Clock::time_point t_submit, t_done;
};

}  // namespace

struct cabs_server {
  int device;
  size_t budget;
  char* pool_base = nullptr;
  Pool* pool = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<uint64_t> slot_req;      // ticket running in each slot (0 = free)
  std::mutex mu;
  std::condition_variable cv;          // wakes the scheduler
  std::condition_variable idle_cv;     // wakes drain()
  std::deque<uint64_t> queue;
  std::map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};
  std::thread worker;
  int running = 0;
};

static void scheduler(cabs_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    bool progressed = false;
    // retire finished slots
    for (size_t k = 0; k < s->streams.size(); ++k) {
      const uint64_t t = s->slot_req[k];
      if (!t) continue;
      if (hipEventQuery(s->events[k]) == hipSuccess) {
        Request& r = s->reqs[t];
        r.t_done = Clock::now();
        r.state = DONE;
        s->pool->release(r.ws_off, r.ws_bytes);
        s->slot_req[k] = 0;
        --s->running;
        progressed = true;
      }
    }
    // admit in arrival order while a slot is free and the workspace fits
    while (!s->queue.empty()) {
      int slot = -1;
      for (size_t k = 0; k < s->streams.size(); ++k)
        if (!s->slot_req[k]) { slot = (int)k; break; }
      if (slot < 0) break;
      const uint64_t t = s->queue.front();
      Request& r = s->reqs[t];
      size_t off;
      if (!s->pool->alloc(r.ws_bytes, off)) break;
      s->queue.pop_front();
      r.ws_off = off;
      r.slot = slot;
      int st = cabs_sketch(&r.mat, &r.prm, s->pool_base + off, r.ws_bytes, &r.res, s->streams[slot]);
      if (st == CABS_OK && r.err_out3)
        st = cabs_error(&r.mat, &r.prm, &r.res, r.err_samples, r.err_seed, s->pool_base + off, r.ws_bytes, r.err_out3,
                        s->streams[slot]);
      if (st != CABS_OK) {
        r.status = st;
        r.state = FAILED;
        r.t_done = Clock::now();
        s->pool->release(off, r.ws_bytes);
        continue;
      }
      (void)hipEventRecord(s->events[slot], s->streams[slot]);
      r.state = RUNNING;
      s->slot_req[slot] = t;
      ++s->running;
      progressed = true;
    }
    if (s->queue.empty() && s->running == 0) s->idle_cv.notify_all();
    if (!progressed) {
      if (s->running > 0) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        s->cv.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
  }
}

extern "C" cabs_server* cabs_server_create(int32_t device, size_t hbm_budget_bytes, int32_t max_slots) {
  if (max_slots < 1 || max_slots > 64 || hbm_budget_bytes < 4096) return nullptr;
  if (hipSetDevice(device) != hipSuccess) return nullptr;
  cabs_server* s = new cabs_server();
  s->device = device;
  s->budget = hbm_budget_bytes;
  if (hipMalloc((void**)&s->pool_base, hbm_budget_bytes) != hipSuccess) {
    delete s;
    return nullptr;
  }
  s->pool = new Pool(hbm_budget_bytes);
  s->streams.resize(max_slots);
  s->events.resize(max_slots);
  s->slot_req.assign(max_slots, 0);
  for (int k = 0; k < max_slots; ++k) {
    (void)hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking);
    (void)hipEventCreateWithFlags(&s->events[k], hipEventDisableTiming);
  }
  s->worker = std::thread(scheduler, s);
  return s;
}

extern "C" cabs_status cabs_submit(cabs_server* s, const cabs_matrix* mat, const cabs_params* prm,
                                   const cabs_result* out, int64_t err_samples, uint64_t err_seed, double* err_out3,
                                   uint64_t* ticket) {
  if (!s || !mat || !prm || !out || !ticket || err_samples < 0) return CABS_EINVAL;
  size_t need = cabs_workspace_bytes(mat, prm);
  if (need == 0) return CABS_EINVAL;
  if (err_out3) {
    const size_t ew = cabs_error_workspace_bytes(mat, prm, err_samples);
    if (ew == 0) return CABS_EINVAL;
    need = ew > need ? ew : need;
  }
  if (need > s->budget) return CABS_ENOMEM;
  if (!out->idx_r || !out->idx_c || !out->C || !out->Rt || !out->Umid) return CABS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  Request r;
  r.ticket = s->next_ticket++;
  r.mat = *mat;
  r.prm = *prm;
  r.res = *out;
  r.err_samples = err_samples;
  r.err_seed = err_seed;
  r.err_out3 = err_out3;
  r.ws_bytes = need;
  r.t_submit = Clock::now();
  s->reqs[r.ticket] = r;
  s->queue.push_back(r.ticket);
  *ticket = r.ticket;
  s->cv.notify_all();
  return CABS_OK;
}

extern "C" cabs_status cabs_poll(cabs_server* s, uint64_t ticket, double* latency_s) {
  if (!s) return CABS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return CABS_EINVAL;
  Request& r = it->second;
  if (r.state == QUEUED || r.state == RUNNING) return CABS_EBUSY;
  cabs_status st = r.state == CANCELED ? CABS_ECANCELED : r.state == FAILED ? (cabs_status)r.status : CABS_OK;
  if (latency_s) *latency_s = std::chrono::duration<double>(r.t_done - r.t_submit).count();
  s->reqs.erase(it);
  return st;
}

extern "C" cabs_status cabs_cancel(cabs_server* s, uint64_t ticket) {
  if (!s) return CABS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return CABS_EINVAL;
  if (it->second.state != QUEUED) return it->second.state == RUNNING ? CABS_EBUSY : CABS_OK;
  for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
    if (*q == ticket) { s->queue.erase(q); break; }
  it->second.state = CANCELED;
  it->second.t_done = Clock::now();
  s->cv.notify_all();
  return CABS_OK;
}

extern "C" cabs_status cabs_server_drain(cabs_server* s) {
  if (!s) return CABS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.notify_all();
  s->idle_cv.wait(lk, [s] { return s->queue.empty() && s->running == 0; });
  return CABS_OK;
}

extern "C" void cabs_server_destroy(cabs_server* s) {
  if (!s) return;
  cabs_server_drain(s);
  s->stop.store(true);
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (size_t k = 0; k < s->streams.size(); ++k) {
    (void)hipStreamSynchronize(s->streams[k]);
    (void)hipStreamDestroy(s->streams[k]);
    (void)hipEventDestroy(s->events[k]);
  }
  (void)hipFree(s->pool_base);
  delete s->pool;
  delete s;
}
