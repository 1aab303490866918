// What the server takes from cabs.hip: same-shape sketches run as one group,
// and the calling thread's error message.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/cabs.h"

namespace cabs {

// True when two requests take the same phases with the same SVD shapes (and neither wants
// the factor form), so that their SVDs can share launches.
bool sketch_groupable(const cabs_params* a, const cabs_params* b);

// G (1..4) sketches, request g on streams[g] with its own workspace: every kernel of request g
// runs on streams[g], except the sketch's FP64 SVDs, which run batched on streams[0] after each
// other stream has recorded join_ev[g] and been waited for; the other streams then wait for
// fork_ev.  The results are bitwise those of cabs_sketch.  status[g] receives each request's
// status; the return value is the first error (the launches made before it stay enqueued).
cabs_status sketch_group(int G, const cabs_matrix* const* mats, const cabs_params* const* prms,
                         cabs_result* const* outs, void* const* ws, const size_t* ws_bytes, const hipStream_t* streams,
                         const hipEvent_t* join_ev, hipEvent_t fork_ev, cabs_status* status);

// Sets the message cabs_last_error returns on this thread.
void set_last_error(const char* msg);

}  // namespace cabs
