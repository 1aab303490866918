// Per-kernel-family event timing (see timing.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace cabs {

enum TimerId { T_ASSIGN = 0, T_EVAL, T_TSGEMM, T_GRAM, T_SVD, T_SNAP, T_CENTROID, T_ERROR, T_COUNT };

// Records an event on `st` when constructed and another when destroyed, if
// timing is enabled; the pair is attributed to kernel family `id`.
struct TimerScope {
  TimerScope(int id, hipStream_t st);
  ~TimerScope();
  int id;
  hipStream_t st;
  hipEvent_t a;
  bool on;
};

}  // namespace cabs
