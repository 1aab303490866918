// Continuous-batching sketch server.
//
// Requests of uneven size arrive from any thread (cabs_submit).  A scheduler
// thread admits them as soon as a slot (a HIP stream) is free and their
// workspace fits in the device pool (serve_core.hpp: arrival order with a
// bounded bypass, so a request that does not fit yet lets smaller ones pass a
// limited number of times), enqueues the whole sketch on the slot's stream,
// and retires it when the completion marker (an event) behind its last kernel
// has fired, returning its workspace to the pool.  Requests in different slots
// run concurrently on the device; each one's kernels only touch its own
// buffers, so its result is the same whether it runs alone or next to others.
//
// With group_max > 1 (cabs_server_set_group; off by default), requests
// admitted in the same round whose sketches have the same shape (the same
// sample sizes, precision and options) run as a group: each on its own slot
// stream, with every FP64 SVD of the sketch batched into one launch for the
// group (group.hpp); the results are bitwise those of the same requests run
// alone.
//
// Ordering: cabs_submit records an event on the caller's stream, and the slot
// stream waits for it before the request's first kernel, so buffers the caller
// wrote (or freed and reused) on its stream before submitting are ready.
//
// The pool is one device allocation made at creation, carved first-fit in
// 256-byte units; nothing is allocated per request.  The server mutex guards
// the bookkeeping only: the ~1000 launches of a sketch are enqueued outside it,
// so cabs_submit and cabs_poll never wait for them.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/cabs.h"
#include "group.hpp"
#include "serve_core.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct ReqData {
  cabs_matrix mat;
  cabs_params prm;
  cabs_result res;
  int64_t err_samples = 0;
  uint64_t err_seed = 0;
  double* err_out3 = nullptr;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
  Clock::time_point t_submit, t_done;
};

}  // namespace

struct cabs_server {
  int device;
  size_t budget;
  char* pool_base = nullptr;
  cabs_serve::Core* core = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;      // completion marker of each slot
  std::vector<hipEvent_t> join_events; // a group member's stream before a shared SVD (and the fork after it)
  int group_max = 1;                   // off by default: see cabs_server_set_group
  std::vector<hipEvent_t> free_events; // "ready" events for reuse
  std::mutex mu;
  std::condition_variable cv;          // wakes the scheduler
  std::condition_variable idle_cv;     // wakes drain()
  std::map<uint64_t, ReqData> data;
  std::atomic<bool> stop{false};
  std::thread worker;
};

static void stamp_done(cabs_server* s, const std::vector<uint64_t>& tickets) {
  const Clock::time_point now = Clock::now();
  for (uint64_t t : tickets) {
    ReqData& d = s->data[t];
    d.t_done = now;
    if (d.ready) {
      s->free_events.push_back(d.ready);
      d.ready = nullptr;
    }
  }
}

static void scheduler(cabs_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop.load()) {
    bool progressed = false;
    std::vector<uint64_t> ret =
        s->core->retire([s](int slot) { return hipEventQuery(s->events[slot]) == hipSuccess; });
    if (!ret.empty()) {
      stamp_done(s, ret);
      progressed = true;
    }
    std::vector<cabs_serve::Launch> adm = s->core->admit();
    if (!adm.empty()) {
      std::vector<ReqData> work;
      work.reserve(adm.size());
      for (const auto& a : adm) work.push_back(s->data[a.ticket]);
      const int gmax = s->group_max;
      lk.unlock();
      std::vector<int> status(adm.size(), CABS_OK);
      std::vector<char> marker(adm.size(), 1);
      // groups of same-shape requests (in admission order)
      std::vector<std::vector<size_t>> groups;
      for (size_t q = 0; q < adm.size(); ++q) {
        bool placed = false;
        for (auto& gset : groups)
          if ((int)gset.size() < gmax && cabs::sketch_groupable(&work[gset[0]].prm, &work[q].prm)) {
            gset.push_back(q);
            placed = true;
            break;
          }
        if (!placed) groups.push_back({q});
      }
      for (const auto& gset : groups) {
        const int G = (int)gset.size();
        std::vector<int> rc(G, CABS_OK);
        for (int g = 0; g < G; ++g) {
          ReqData& r = work[gset[g]];
          if (r.ready && hipStreamWaitEvent(s->streams[adm[gset[g]].slot], r.ready, 0) != hipSuccess)
            rc[g] = CABS_EDEVICE;
        }
        bool all_ok = true;
        for (int g = 0; g < G; ++g) all_ok = all_ok && rc[g] == CABS_OK;
        if (G == 1) {
          const size_t q = gset[0];
          ReqData& r = work[q];
          if (rc[0] == CABS_OK)
            rc[0] = cabs_sketch(&r.mat, &r.prm, s->pool_base + adm[q].off, adm[q].bytes, &r.res,
                                s->streams[adm[q].slot]);
        } else if (all_ok) {
          const cabs_matrix* mats[4];
          const cabs_params* prms[4];
          cabs_result* outs[4];
          void* wss[4];
          size_t wsb[4];
          hipStream_t sts[4];
          hipEvent_t jev[4];
          cabs_status gst[4];
          for (int g = 0; g < G; ++g) {
            const size_t q = gset[g];
            mats[g] = &work[q].mat;
            prms[g] = &work[q].prm;
            outs[g] = &work[q].res;
            wss[g] = s->pool_base + adm[q].off;
            wsb[g] = adm[q].bytes;
            sts[g] = s->streams[adm[q].slot];
            jev[g] = s->join_events[adm[q].slot];
            gst[g] = CABS_OK;
          }
          const cabs_status grc = cabs::sketch_group(G, mats, prms, outs, wss, wsb, sts, jev, jev[0], gst);
          for (int g = 0; g < G; ++g) rc[g] = gst[g] != CABS_OK ? gst[g] : grc;
        }
        for (int g = 0; g < G; ++g) {
          const size_t q = gset[g];
          ReqData& r = work[q];
          hipStream_t st = s->streams[adm[q].slot];
          void* ws = s->pool_base + adm[q].off;
          if (rc[g] == CABS_OK && r.err_out3)
            rc[g] = cabs_error(&r.mat, &r.prm, &r.res, r.err_samples, r.err_seed, ws, adm[q].bytes, r.err_out3, st);
          // The marker goes behind whatever was enqueued, also after an error: kernels queued before
          // it may still run, so the workspace stays held until the marker has fired.
          if (hipEventRecord(s->events[adm[q].slot], st) != hipSuccess) {
            (void)hipStreamSynchronize(st);
            marker[q] = 0;
            if (rc[g] == CABS_OK) rc[g] = CABS_EDEVICE;
          }
          status[q] = rc[g];
        }
      }
      lk.lock();
      std::vector<uint64_t> ended;
      for (size_t q = 0; q < adm.size(); ++q) {
        s->core->launched(adm[q].ticket, status[q], marker[q] != 0);
        if (!marker[q]) ended.push_back(adm[q].ticket);
      }
      stamp_done(s, ended);
      progressed = true;
    }
    if (s->core->idle()) s->idle_cv.notify_all();
    if (!progressed) {
      if (s->core->running() > 0) {
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
  if (max_slots < 1 || max_slots > 64 || hbm_budget_bytes < 4096) {
    cabs::set_last_error("cabs_server_create: max_slots must be 1..64 and the budget at least 4096 bytes");
    return nullptr;
  }
  if (hipSetDevice(device) != hipSuccess) {
    cabs::set_last_error("cabs_server_create: hipSetDevice failed");
    return nullptr;
  }
  cabs_server* s = new cabs_server();
  s->device = device;
  s->budget = hbm_budget_bytes;
  if (hipMalloc((void**)&s->pool_base, hbm_budget_bytes) != hipSuccess) {
    cabs::set_last_error("cabs_server_create: the memory pool could not be allocated");
    delete s;
    return nullptr;
  }
  s->core = new cabs_serve::Core(hbm_budget_bytes, max_slots, 4 * max_slots);
  s->streams.resize(max_slots);
  s->events.resize(max_slots);
  s->join_events.resize(max_slots);
  // a slot's stream and events, or none of the server if one cannot be made
  bool made = true;
  for (int k = 0; k < max_slots && made; ++k) {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr, join = nullptr;
    made = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    if (made) s->streams[k] = st;
    made = made && hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess;
    if (made) s->events[k] = done;
    made = made && hipEventCreateWithFlags(&join, hipEventDisableTiming) == hipSuccess;
    if (made) s->join_events[k] = join;
  }
  if (!made) {
    cabs::set_last_error("cabs_server_create: a slot's stream or events could not be created");
    for (int k = 0; k < max_slots; ++k) {
      if (s->streams[k]) (void)hipStreamDestroy(s->streams[k]);
      if (s->events[k]) (void)hipEventDestroy(s->events[k]);
      if (s->join_events[k]) (void)hipEventDestroy(s->join_events[k]);
    }
    (void)hipFree(s->pool_base);
    delete s->core;
    delete s;
    return nullptr;
  }
  s->worker = std::thread(scheduler, s);
  return s;
}

extern "C" cabs_status cabs_submit(cabs_server* s, const cabs_matrix* mat, const cabs_params* prm,
                                   const cabs_result* out, int64_t err_samples, uint64_t err_seed, double* err_out3,
                                   void* stream, uint64_t* ticket) {
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
  hipEvent_t ev = nullptr;
  if (!s->free_events.empty()) {
    ev = s->free_events.back();
    s->free_events.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    return CABS_EDEVICE;
  }
  if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
    s->free_events.push_back(ev);
    return CABS_EDEVICE;
  }
  const uint64_t t = s->core->submit(need);
  if (t == 0) {
    s->free_events.push_back(ev);
    return CABS_ENOMEM;
  }
  ReqData r;
  r.mat = *mat;
  r.prm = *prm;
  r.res = *out;
  r.err_samples = err_samples;
  r.err_seed = err_seed;
  r.err_out3 = err_out3;
  r.ready = ev;
  r.t_submit = Clock::now();
  s->data[t] = r;
  *ticket = t;
  s->cv.notify_all();
  return CABS_OK;
}

extern "C" cabs_status cabs_poll(cabs_server* s, uint64_t ticket, double* latency_s) {
  if (!s) return CABS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  const cabs_serve::Entry* e = s->core->find(ticket);
  if (!e) return CABS_EINVAL;
  if (e->state == cabs_serve::QUEUED || e->state == cabs_serve::LAUNCHING || e->state == cabs_serve::RUNNING)
    return CABS_EBUSY;
  const cabs_status st = e->state == cabs_serve::CANCELED ? CABS_ECANCELED
                         : e->state == cabs_serve::FAILED ? (cabs_status)e->status
                                                          : CABS_OK;
  ReqData& d = s->data[ticket];
  if (latency_s) *latency_s = std::chrono::duration<double>(d.t_done - d.t_submit).count();
  if (d.ready) s->free_events.push_back(d.ready);
  s->data.erase(ticket);
  s->core->forget(ticket);
  return st;
}

extern "C" cabs_status cabs_cancel(cabs_server* s, uint64_t ticket) {
  if (!s) return CABS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  const int rc = s->core->cancel(ticket);
  if (rc < 0) return CABS_EINVAL;
  if (rc > 0) return CABS_EBUSY;
  auto it = s->data.find(ticket);
  if (it != s->data.end() && it->second.t_done == Clock::time_point()) it->second.t_done = Clock::now();
  s->cv.notify_all();
  return CABS_OK;
}

extern "C" cabs_status cabs_server_set_group(cabs_server* s, int32_t group_max) {
  if (!s || group_max < 1 || group_max > 4) return CABS_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  s->group_max = group_max;
  return CABS_OK;
}

extern "C" cabs_status cabs_server_drain(cabs_server* s) {
  if (!s) return CABS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv.notify_all();
  s->idle_cv.wait(lk, [s] { return s->core->idle(); });
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
    (void)hipEventDestroy(s->join_events[k]);
  }
  for (auto& kv : s->data)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  (void)hipFree(s->pool_base);
  delete s->core;
  delete s;
}
