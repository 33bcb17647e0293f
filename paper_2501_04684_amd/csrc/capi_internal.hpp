// Internal declarations shared by the C ABI sources (not installed).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "../../include/ubf.h"
#include "plan.hpp"

struct ubf_plan {
  ubf::Plan p;
  // Stage timing (ubf_profile_begin/end): a start and a stop event per
  // stage of each recorded call, one call in prof_every recorded.
  static constexpr size_t kEventsPerCall = 6;
  std::vector<hipEvent_t> events;
  int32_t prof_max = 0;
  int32_t prof_n = 0;
  int32_t prof_every = 1;
  int64_t prof_seen = 0;
  bool profiling = false;
  // Captured three-stage product (ubf_plan_capture / ubf_plan_replay).
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  // Events for the next recorded product, or NULL when not profiling.
  hipEvent_t* next_events() {
    if (!profiling || prof_n >= prof_max) return nullptr;
    if (prof_seen++ % prof_every != 0) return nullptr;
    return &events[kEventsPerCall * (size_t)prof_n++];
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~ubf_plan() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace ubf {

// Error reporting: set the thread-local message and return the status.
int fail(int status, const std::string& why);
int ok();
int hip_fail(int err, const char* what);
const std::string& last_error_text();

// Argument checks shared by the compute entry points (null pointers, an
// unbound plan, nrhs outside 1..max_nrhs, overlapping input and output);
// nothing touches a device.
int check_call(ubf_plan* plan, const void* in, void* out, int32_t nrhs, size_t in_bytes,
               size_t out_bytes);
// Bytes of [nrhs][sum N_b] complex64 (the product's x and y).
size_t basis_vec_bytes(const Plan& p, int32_t nrhs);

// The three stages of the product y = T G S x, enqueued on `s`
// (ev: optional timing events, a start and a stop per stage).
int enqueue_mvm(const Plan& p, const void* d_x, void* d_y, int32_t nrhs, hipStream_t s,
                hipEvent_t* ev);

}  // namespace ubf
