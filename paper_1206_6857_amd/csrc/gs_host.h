// Host-side declarations shared by the C ABI and the orchestration code.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/gausssum.h"
#include "gs_policy.h"

namespace gs {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

struct gs_ctx_base;

// Named device buffers, grown geometrically and reused across calls.
struct Workspace {
  std::map<std::string, Buf> bufs;
  std::map<std::string, Buf> pinned;  // page-locked host buffers (hipHostMalloc)
  void* get(const std::string& name, size_t bytes, gs_ctx_base* ctx, hipError_t* err);
  void* get_pinned(const std::string& name, size_t bytes, hipError_t* err);
  void release(const std::string& name);  // frees one named device buffer (no-op if absent)
  void release_all();
};

// Host copy of a kd-tree, kept for introspection when keep_trace is set.
struct HostTree {
  bool valid = false;
  int64_t n_nodes = 0, n_points = 0;
  std::vector<int32_t> perm, begin, count, left;
  std::vector<double> lo, hi, ctr, rinf, W, wmin, rad;
};

// A recorded pair of timing events not yet read (see KernelTimer).
struct PendingTimer {
  hipEvent_t a, b;
  int cls, launches;
};

struct gs_ctx_base {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // A side stream (default priority) for work that is independent of the
  // base cases: forked from `stream` with fork_ev, joined with join_ev.
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  std::string err;
  gs_stats stats;
  Workspace ws;
  std::vector<int64_t> pair_counts;   // [n_h][6]
  std::vector<int32_t> trace;         // [n][6]
  std::vector<float> trace_feat;      // [n][16] pair features (policy logging)
  std::vector<int16_t> trace_feas;    // [n] admitted orders (policy logging)
  HostTree host_tree[2];
  bool kernel_timing = false;
  unsigned timing_mask = 0;  // kernel classes (bit GS_K_*) timed by KernelTimer
  PolicyState policy;
  std::map<std::string, std::pair<int, int>> tuned;  // autotuner: signature -> (method, leaf)
  std::vector<hipEvent_t> ev_pool;                    // reusable timing events
  // Error-path testing (gs_options.debug_fail_alloc): the device workspace
  // request that fails (0: none), the requests of the current call so far,
  // and the nesting depth of the API calls that armed them.
  int64_t fail_alloc_at = 0, alloc_requests = 0;
  int alloc_scope = 0;
  // Counts one device workspace request; true when it is the one to fail.
  bool inject_alloc_failure() { return ++alloc_requests == fail_alloc_at; }
  // decision counters of the last dual-tree call, being copied to pinned
  // memory; read by finish_dualtree_stats once the stream has drained
  const unsigned long long* stats_pending = nullptr;
  int stats_pending_nh = 0;
  std::vector<PendingTimer> pending;                  // recorded, not yet read
};

// Staged, validated inputs in device memory.
struct DeviceInputs {
  int64_t M = 0, N = 0;
  int D = 0;
  bool mono = false;
  double* q_soa = nullptr;  // [D][M]
  double* q_aos = nullptr;  // [M][D]
  double* r_soa = nullptr;  // [D][N]
  double* r_aos = nullptr;  // [N][D]
  double* w = nullptr;      // [N]
};

bool is_device_pointer(const void* p);

// Optional HIP-event timing of one kernel class on the context's stream:
// construct before the launches, call stop() after them.  No synchronisation:
// the events are read by flush_kernel_timers (end of the call), which adds
// the elapsed device time to stats.k_ms[cls].
struct KernelTimer {
  gs_ctx_base* ctx = nullptr;
  int cls = 0;
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  KernelTimer(gs_ctx_base* c, bool enabled, int k, hipStream_t s);
  void stop(hipStream_t s, int n_launches);
  ~KernelTimer();
};
void flush_kernel_timers(gs_ctx_base* ctx);

// Graded multi-index set with |alpha| < p (section 2), library order.
std::vector<std::vector<int>> multi_indices(int D, int p);
// alpha with every alpha_d < p, by largest component (O(p^D) expansions)
std::vector<std::vector<int>> tensor_indices(int D, int p);
// own_exp(x), x / y and sqrt(y) elementwise into out[3][n] (device pointers; k_decide.hip).
hipError_t launch_decision_arith(const double* x, const double* y, int64_t n, double* out, hipStream_t s);
// order limit of the O(p^D) expansions for dimension D
int plimit_tensor(int D);

// Learned pair policy (policy.cpp).
void policy_default_costs(PolicyState& ps);
gs_status policy_device_model(gs_ctx_base* ctx, PolicyDevModel* m);
void policy_calibrate_costs(gs_ctx_base* ctx, int D);
gs_status policy_build_records(gs_ctx_base* ctx, int D, const std::vector<double>& hs);
gs_status policy_train(gs_ctx_base* ctx, const float* rec, int64_t n, const gs_train_opts& o,
                       float* final_loss);
gs_status policy_gradient(gs_ctx_base* ctx, const float* rec, int64_t n, float* grad, float* loss);
gs_status policy_predict(gs_ctx_base* ctx, const float* feat, int64_t n, float* scores);
int64_t policy_param_floats();
void policy_get_params(const PolicyState& ps, float* out);
gs_status policy_set_params(gs_ctx_base* ctx, const float* in);
gs_status policy_save(gs_ctx_base* ctx, const char* path);
gs_status policy_load(gs_ctx_base* ctx, const char* path);
gs_status policy_write_log(gs_ctx_base* ctx, const char* path);
gs_status policy_read_log(gs_ctx_base* ctx, const char* path, std::vector<float>* rec);

// Folds the counters of the last dual-tree call into stats and pair_counts;
// the stream must have drained.
void finish_dualtree_stats(gs_ctx_base* ctx);

// Dual-tree summation (GS_DUALTREE, GS_DFD, GS_DFDO) into G_dev[n_h][M].
gs_status run_dualtree(gs_ctx_base* ctx, const DeviceInputs& in, const std::vector<double>& hs,
                       double eps, const gs_options& opt, double* G_dev);

}  // namespace gs
