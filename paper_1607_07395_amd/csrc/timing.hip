// Optional per-kernel-family timing with HIP events recorded on the launch
// stream (diagnostics for roofline figures).  Disabled by default; when
// disabled a TimerScope costs one relaxed atomic load.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/cabs.h"
#include "timing.hpp"

namespace cabs {

static std::atomic<int> g_timing_on{0};
static std::mutex g_timing_mu;
struct Rec { int id; hipEvent_t a, b; };
static std::vector<Rec> g_recs;
static std::vector<hipEvent_t> g_free;

static const char* kNames[T_COUNT] = {"assign", "eval", "tsgemm", "gram", "svd", "snap", "centroid", "error"};

static hipEvent_t take_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

TimerScope::TimerScope(int id_, hipStream_t st_) : id(id_), st(st_), a(nullptr), on(false) {
  if (!g_timing_on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> g(g_timing_mu);
  a = take_event();
  if (a && hipEventRecord(a, st) == hipSuccess) on = true;
}

TimerScope::~TimerScope() {
  if (!on) return;
  std::lock_guard<std::mutex> g(g_timing_mu);
  hipEvent_t b = take_event();
  if (b && hipEventRecord(b, st) == hipSuccess) g_recs.push_back({id, a, b});
}

}  // namespace cabs

using namespace cabs;

extern "C" cabs_status cabs_timing_enable(int32_t on) {
  g_timing_on.store(on ? 1 : 0);
  return CABS_OK;
}

extern "C" void cabs_timing_reset(void) {
  std::lock_guard<std::mutex> g(g_timing_mu);
  for (auto& r : g_recs) {
    (void)hipEventSynchronize(r.b);
    g_free.push_back(r.a);
    g_free.push_back(r.b);
  }
  g_recs.clear();
}

extern "C" cabs_status cabs_timing_read(const char* family, double* total_ms, int64_t* launches) {
  if (!family || !total_ms || !launches) return CABS_EINVAL;
  int id = -1;
  for (int i = 0; i < T_COUNT; ++i)
    if (std::strcmp(family, kNames[i]) == 0) id = i;
  if (id < 0) return CABS_EINVAL;
  std::lock_guard<std::mutex> g(g_timing_mu);
  double tot = 0.0;
  int64_t n = 0;
  for (auto& r : g_recs) {
    if (r.id != id) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return CABS_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return CABS_EDEVICE;
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  return CABS_OK;
}
