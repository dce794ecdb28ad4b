// The plan object shared by the C ABI (abac_api.hip) and the request server
// (server.hip).  Internal: not part of the public header.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/abac.h"
#include "abac_internal.h"

using abac::DevPlan;
using abac::MinresState;
using abac::kSnapRing;

struct ProfPair {
  int kid;
  hipEvent_t e0, e1;
};


struct abac_plan {
  DevPlan P;
  int prec;
  double T, alpha;
  hipStream_t stream;
  void* ws;
  size_t ws_bytes;
  bool own_ws;
  // variable-coefficient face weights (workspace region) and the preconditioner's
  // constant coefficient abar (1 for the constant-coefficient problem)
  double* coef_ws;
  double abar;
  // asynchronous solve bookkeeping
  MinresState* h_ring;   // host-mapped pinned memory, kSnapRing * B states written by the device
  hipEvent_t ring_ev[kSnapRing];
  long long ring_posted;  // snapshots enqueued in the current solve (= device sequence number)
  const double* f;
  double* u;
  bool active;
  // one MINRES iteration captured as a graph (launched on the plan stream)
  bool use_graph;
  hipStream_t cap_stream;
  hipGraphExec_t iter_graph;
  const double* graph_f;
  double* graph_u;
  // kernel timing
  bool prof;
  std::vector<ProfPair> pending;
  std::vector<hipEvent_t> event_pool;
  double prof_ms[ABAC_K_COUNT];
  long long prof_n[ABAC_K_COUNT];
};

namespace abac {
// Non-blocking: if snapshot `seq` of the current solve has been written, set *ready
// and return a pointer to its per-RHS states (host memory); otherwise *ready = 0.
abac_status plan_peek_snapshot(abac_plan* p, long long seq, int* ready, const MinresState** states);
// Number of snapshots enqueued in the current solve (the set-up one is number 0).
long long plan_snapshots_posted(const abac_plan* p);
hipError_t launch_fill_normal(double* out, unsigned long long n, unsigned long long seed, hipStream_t s);
hipError_t launch_fill_zero(double* out, unsigned long long n, hipStream_t s);
// the thread-local message abac_last_error() returns
void set_last_error(const std::string& msg);
// whether a group (abac_group_set) can take the plan as a member (its solve aside)
bool group_accepts(const abac_plan* p);
}  // namespace abac
