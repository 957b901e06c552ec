// Host-side declarations shared by the C ABI and the orchestration code.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/gausssum.h"

namespace gs {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

struct gs_ctx_base;

// Named device buffers, grown geometrically and reused across calls.
struct Workspace {
  std::map<std::string, Buf> bufs;
  void* get(const std::string& name, size_t bytes, gs_ctx_base* ctx, hipError_t* err);
  void release_all();
};

// Host copy of a kd-tree, kept for introspection when keep_trace is set.
struct HostTree {
  bool valid = false;
  int64_t n_nodes = 0, n_points = 0;
  std::vector<int32_t> perm, begin, count, left;
  std::vector<double> lo, hi, ctr, rinf, W, wmin;
};

struct gs_ctx_base {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  gs_stats stats;
  Workspace ws;
  std::vector<int64_t> pair_counts;   // [n_h][6]
  std::vector<int32_t> trace;         // [n][6]
  HostTree host_tree[2];
  bool kernel_timing = false;
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
// construct before the launches, call stop() after them; the elapsed device
// time is added to stats.k_ms[cls] once the stream is synchronised (flush()).
struct KernelTimer {
  gs_ctx_base* ctx = nullptr;
  int cls = 0;
  int launches = 0;
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  KernelTimer(gs_ctx_base* c, bool enabled, int k, hipStream_t s);
  void stop(hipStream_t s, int n_launches);
  ~KernelTimer();
};

// Graded multi-index set with |alpha| < p (section 2), library order.
std::vector<std::vector<int>> multi_indices(int D, int p);

// Dual-tree summation (GS_DUALTREE, GS_DFD, GS_DFDO) into G_dev[n_h][M].
gs_status run_dualtree(gs_ctx_base* ctx, const DeviceInputs& in, const std::vector<double>& hs,
                       double eps, const gs_options& opt, double* G_dev);

}  // namespace gs
