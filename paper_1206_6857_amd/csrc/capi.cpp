// C ABI entry points: argument validation, staging of caller buffers, device
// workspace, and orchestration of the kernels of the other translation units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/gausssum.h"
#include "gs_internal.h"
#include "gs_host.h"

using namespace gs;

// ------------------------------------------------------------------ helpers

namespace gs {

void* Workspace::get(const std::string& name, size_t bytes, gs_ctx_base* ctx, hipError_t* err) {
  if (ctx && ctx->inject_alloc_failure()) {
    *err = hipErrorOutOfMemory;
    return nullptr;
  }
  Buf& b = bufs[name];
  if (bytes == 0) bytes = 16;
  if (b.cap < bytes) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    size_t cap = std::max(bytes, b.cap + b.cap / 2);
    hipError_t e = hipMalloc(&b.p, cap);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      b.cap = 0;
      *err = e;
      return nullptr;
    }
    b.cap = cap;
  }
  return b.p;
}

void* Workspace::get_pinned(const std::string& name, size_t bytes, hipError_t* err) {
  Buf& b = pinned[name];
  if (bytes == 0) bytes = 16;
  if (b.cap < bytes) {
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    size_t cap = std::max(bytes, b.cap + b.cap / 2);
    hipError_t e = hipHostMalloc(&b.p, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      b.cap = 0;
      *err = e;
      return nullptr;
    }
    b.cap = cap;
  }
  return b.p;
}

void Workspace::release(const std::string& name) {
  auto it = bufs.find(name);
  if (it == bufs.end()) return;
  if (it->second.p) (void)hipFree(it->second.p);
  bufs.erase(it);
}

void Workspace::release_all() {
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  bufs.clear();
  for (auto& kv : pinned)
    if (kv.second.p) (void)hipHostFree(kv.second.p);
  pinned.clear();
}

bool is_device_pointer(const void* p) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

static hipEvent_t pooled_event(gs_ctx_base* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

KernelTimer::KernelTimer(gs_ctx_base* c, bool enabled, int k, hipStream_t s) : ctx(c), cls(k) {
  if (!enabled || !((c->timing_mask >> k) & 1u)) return;
  a = pooled_event(ctx);
  b = pooled_event(ctx);
  if (!a || !b) return;
  on = hipEventRecord(a, s) == hipSuccess;
}

void KernelTimer::stop(hipStream_t s, int n_launches) {
  if (!on) return;
  on = false;
  if (hipEventRecord(b, s) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  ctx->pending.push_back({a, b, cls, n_launches});
  a = b = nullptr;  // owned by the pending list now
}

KernelTimer::~KernelTimer() {
  if (a) ctx->ev_pool.push_back(a);
  if (b) ctx->ev_pool.push_back(b);
}

void flush_kernel_timers(gs_ctx_base* ctx) {
  for (const PendingTimer& p : ctx->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->stats.k_ms[p.cls] += ms;
      ctx->stats.k_launches[p.cls] += p.launches;
    } else {
      (void)hipGetLastError();
    }
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

}  // namespace gs

struct gs_ctx : gs::gs_ctx_base {};

#define GS_FAIL(ctx, code, msg)    \
  do {                             \
    (ctx)->err = (msg);            \
    return (code);                 \
  } while (0)

#define GS_HIP(ctx, call)                                                             \
  do {                                                                                \
    hipError_t _e = (call);                                                           \
    if (_e != hipSuccess) {                                                           \
      (void)hipGetLastError();                                                        \
      (ctx)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(_e); \
      return _e == hipErrorOutOfMemory ? GS_ENOMEM : GS_EDEVICE;                      \
    }                                                                                 \
  } while (0)

template <class T>
static T* wsget(gs_ctx* ctx, const char* name, size_t count, gs_status* st) {
  hipError_t e = hipSuccess;
  void* p = ctx->ws.get(name, count * sizeof(T), ctx, &e);
  if (!p) {
    ctx->err = std::string("device allocation failed for workspace '") + name + "' (" +
               std::to_string(count * sizeof(T)) + " bytes): " + hipGetErrorString(e);
    *st = GS_ENOMEM;
  }
  return static_cast<T*>(p);
}

#define WS(T, name, count)                          \
  ({                                                \
    gs_status _st = GS_OK;                          \
    T* _p = wsget<T>(ctx, name, (size_t)(count), &_st); \
    if (!_p) return _st;                            \
    _p;                                             \
  })

// Arms gs_options.debug_fail_alloc for the outermost API call and disarms it
// when that call returns; a nested call (gs_lscv's sum) shares the count.
struct AllocFaultScope {
  gs_ctx* c;
  AllocFaultScope(gs_ctx* ctx, int32_t k) : c(ctx) {
    if (c->alloc_scope++ == 0) {
      c->fail_alloc_at = k;
      c->alloc_requests = 0;
    }
  }
  ~AllocFaultScope() {
    if (--c->alloc_scope == 0) c->fail_alloc_at = 0;
  }
};

// A call that fails after it enqueued work drains both streams before it
// returns, so that none of its kernels still reads the caller's buffers or
// the workspace when the caller frees the one or reuses the other.
struct DrainOnFailure {
  gs_ctx* c;
  bool ok = false;
  ~DrainOnFailure() {
    if (ok) return;
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamSynchronize(c->stream);
    (void)hipGetLastError();
  }
};

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ C ABI

extern "C" {

void gs_default_options(gs_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->struct_size = (int32_t)sizeof(gs_options);
  opt->leaf_size = 64;
  opt->plimit = 0;
  opt->method = GS_DUALTREE;
  opt->policy = GS_RULE;
  opt->monochromatic = -1;
  opt->blocking = 1;
  opt->keep_trace = 0;
  opt->log_pairs = 0;
  opt->eps_round_share = 0.1;
}

gs_status gs_create(gs_ctx** out, int32_t device, void* hip_stream) {
  if (!out) return GS_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return GS_EDEVICE;
  }
  gs_ctx* ctx = new (std::nothrow) gs_ctx();
  if (!ctx) return GS_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete ctx;
    return GS_EDEVICE;
  }
  if (hip_stream) {
    ctx->stream = (hipStream_t)hip_stream;
    ctx->own_stream = false;
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return GS_EDEVICE;
    }
    ctx->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return GS_EDEVICE;
  }
  std::memset(&ctx->stats, 0, sizeof(ctx->stats));
  policy_default_costs(ctx->policy);
  *out = ctx;
  return GS_OK;
}

gs_status gs_destroy(gs_ctx* ctx) {
  if (!ctx) return GS_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  flush_kernel_timers(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  ctx->ev_pool.clear();
  (void)hipStreamSynchronize(ctx->side);
  (void)hipStreamDestroy(ctx->side);
  (void)hipEventDestroy(ctx->fork_ev);
  (void)hipEventDestroy(ctx->join_ev);
  ctx->ws.release_all();
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return GS_OK;
}

const char* gs_last_error(gs_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

// Pending counters and timers of a non-blocking call: drain the stream first.
static void settle(gs_ctx* ctx) {
  if (!ctx->stats_pending && ctx->pending.empty()) return;
  (void)hipSetDevice(ctx->device);
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) (void)hipGetLastError();
  finish_dualtree_stats(ctx);
  flush_kernel_timers(ctx);
}

gs_status gs_get_stats(gs_ctx* ctx, gs_stats* out) {
  if (!ctx || !out) return GS_EINVAL;
  settle(ctx);
  if (out->struct_size < (int32_t)sizeof(gs_stats)) GS_FAIL(ctx, GS_EINVAL, "gs_stats.struct_size too small");
  *out = ctx->stats;
  out->struct_size = (int32_t)sizeof(gs_stats);
  return GS_OK;
}

gs_status gs_get_pair_counts(gs_ctx* ctx, int64_t* counts) {
  if (!ctx || !counts) return GS_EINVAL;
  settle(ctx);
  std::copy(ctx->pair_counts.begin(), ctx->pair_counts.end(), counts);
  return GS_OK;
}

gs_status gs_get_tree(gs_ctx* ctx, int32_t which, int64_t* n_nodes, int64_t* n_points,
                      int32_t* perm, int32_t* begin, int32_t* count, int32_t* left, double* lo,
                      double* hi, double* ctr, double* rinf, double* W, double* wmin, double* rad) {
  if (!ctx || which < 0 || which > 1) return GS_EINVAL;
  const HostTree& t = ctx->host_tree[which];
  if (!t.valid) GS_FAIL(ctx, GS_EINVAL, "no tree kept: call gauss_sum with keep_trace = 1 first");
  if (n_nodes) *n_nodes = t.n_nodes;
  if (n_points) *n_points = t.n_points;
  auto cp = [](auto* dst, const auto& v) {
    if (dst) std::copy(v.begin(), v.end(), dst);
  };
  cp(perm, t.perm);
  cp(begin, t.begin);
  cp(count, t.count);
  cp(left, t.left);
  cp(lo, t.lo);
  cp(hi, t.hi);
  cp(ctr, t.ctr);
  cp(rinf, t.rinf);
  cp(W, t.W);
  cp(wmin, t.wmin);
  if (rad) {
    if (t.rad.size() == (size_t)t.n_nodes)
      cp(rad, t.rad);
    else
      std::fill(rad, rad + t.n_nodes, 0.0);
  }
  return GS_OK;
}

gs_status gs_multi_indices(int32_t D, int32_t p, int64_t* n_terms, int32_t* alpha) {
  if (D < 1 || D > kMaxD || p < 1 || p > kMaxPlimit || !n_terms) return GS_EINVAL;
  auto mis = multi_indices(D, p);
  *n_terms = (int64_t)mis.size();
  if (alpha)
    for (size_t i = 0; i < mis.size(); ++i)
      for (int d = 0; d < D; ++d) alpha[i * D + d] = mis[i][d];
  return GS_OK;
}

gs_status gs_tensor_indices(int32_t D, int32_t p, int64_t* n_terms, int32_t* alpha) {
  if (D < 1 || D > kMaxD || p < 1 || p > kMaxPlimit || !n_terms) return GS_EINVAL;
  double terms = 1.0;
  for (int d = 0; d < D; ++d) terms *= p;
  if (terms > (double)kMaxTerms) return GS_EINVAL;
  auto mis = tensor_indices(D, p);
  *n_terms = (int64_t)mis.size();
  if (alpha)
    for (size_t i = 0; i < mis.size(); ++i)
      for (int d = 0; d < D; ++d) alpha[i * D + d] = mis[i][d];
  return GS_OK;
}

gs_status gs_decision_arith(gs_ctx* ctx, const double* x, const double* y, int64_t n, double* out) {
  if (!ctx) return GS_EINVAL;
  ctx->err.clear();
  if (!x || !y || !out) GS_FAIL(ctx, GS_EINVAL, "null array pointer");
  if (n < 1 || n > (int64_t)1 << 24) GS_FAIL(ctx, GS_EINVAL, "n must be in [1, 2^24]");
  GS_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  // a test entry point: its buffers (up to 640 MiB) are freed when it returns
  struct Release {
    gs_ctx* c;
    ~Release() {
      (void)hipStreamSynchronize(c->stream);
      c->ws.release("arith_x");
      c->ws.release("arith_y");
      c->ws.release("arith_out");
    }
  } release{ctx};
  double* dx = WS(double, "arith_x", n);
  double* dy = WS(double, "arith_y", n);
  double* dout = WS(double, "arith_out", 3 * n);
  GS_HIP(ctx, hipMemcpyAsync(dx, x, n * sizeof(double), hipMemcpyHostToDevice, st));
  GS_HIP(ctx, hipMemcpyAsync(dy, y, n * sizeof(double), hipMemcpyHostToDevice, st));
  GS_HIP(ctx, launch_decision_arith(dx, dy, n, dout, st));
  GS_HIP(ctx, hipMemcpyAsync(out, dout, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
  GS_HIP(ctx, hipStreamSynchronize(st));
  return GS_OK;
}

void gs_default_train_opts(gs_train_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int32_t)sizeof(gs_train_opts);
  o->steps = 3000;
  o->batch = 4096;
  o->reinit = 1;
  o->seed = 1;
  o->lr = 2e-3;
}

gs_status gs_policy_set_cost_model(gs_ctx* ctx, const gs_cost_model* cm) {
  if (!ctx || !cm) return GS_EINVAL;
  const double v[5] = {cm->pair_ns, cm->dh_ns, cm->dl_ns, cm->h2l_ns, cm->base_ns};
  for (double x : v)
    if (!(x >= 0.0) || !std::isfinite(x)) GS_FAIL(ctx, GS_EINVAL, "cost model entries must be finite and >= 0");
  PolicyState& ps = ctx->policy;
  ps.c_pair = v[0];
  ps.c_dh = v[1];
  ps.c_dl = v[2];
  ps.c_h2l = v[3];
  ps.c_base = v[4];
  ps.costs_pinned = true;
  return GS_OK;
}

gs_status gs_policy_get_cost_model(gs_ctx* ctx, gs_cost_model* cm) {
  if (!ctx || !cm) return GS_EINVAL;
  const PolicyState& ps = ctx->policy;
  cm->pair_ns = ps.c_pair;
  cm->dh_ns = ps.c_dh;
  cm->dl_ns = ps.c_dl;
  cm->h2l_ns = ps.c_h2l;
  cm->base_ns = ps.c_base;
  return GS_OK;
}

gs_status gs_policy_get_log(gs_ctx* ctx, int64_t* n_records, float* records, int32_t* keys) {
  if (!ctx || !n_records) return GS_EINVAL;
  const PolicyState& ps = ctx->policy;
  *n_records = (int64_t)(ps.log.size() / kPolicyRecord);
  if (records) std::copy(ps.log.begin(), ps.log.end(), records);
  if (keys) std::copy(ps.log_keys.begin(), ps.log_keys.end(), keys);
  return GS_OK;
}

gs_status gs_policy_write_log(gs_ctx* ctx, const char* path) {
  if (!ctx || !path) return GS_EINVAL;
  ctx->err.clear();
  return policy_write_log(ctx, path);
}

static gs_status train_opts_of(gs_ctx* ctx, const gs_train_opts* in, gs_train_opts* o) {
  gs_default_train_opts(o);
  if (in) {
    if (in->struct_size != (int32_t)sizeof(gs_train_opts))
      GS_FAIL(ctx, GS_EINVAL, "gs_train_opts.struct_size does not match this library");
    *o = *in;
  }
  return GS_OK;
}

gs_status gs_policy_train(gs_ctx* ctx, const char* log_path, const gs_train_opts* opts, float* final_loss) {
  if (!ctx || !log_path) return GS_EINVAL;
  ctx->err.clear();
  gs_train_opts o;
  gs_status s = train_opts_of(ctx, opts, &o);
  if (s != GS_OK) return s;
  std::vector<float> rec;
  s = policy_read_log(ctx, log_path, &rec);
  if (s != GS_OK) return s;
  GS_HIP(ctx, hipSetDevice(ctx->device));
  return policy_train(ctx, rec.data(), (int64_t)(rec.size() / kPolicyRecord), o, final_loss);
}

gs_status gs_policy_train_records(gs_ctx* ctx, const float* records, int64_t n, const gs_train_opts* opts,
                                  float* final_loss) {
  if (!ctx || !records) return GS_EINVAL;
  ctx->err.clear();
  gs_train_opts o;
  gs_status s = train_opts_of(ctx, opts, &o);
  if (s != GS_OK) return s;
  GS_HIP(ctx, hipSetDevice(ctx->device));
  return policy_train(ctx, records, n, o, final_loss);
}

gs_status gs_policy_gradient(gs_ctx* ctx, const float* records, int64_t n, float* grad, float* loss) {
  if (!ctx || !records) return GS_EINVAL;
  ctx->err.clear();
  GS_HIP(ctx, hipSetDevice(ctx->device));
  return policy_gradient(ctx, records, n, grad, loss);
}

gs_status gs_policy_predict(gs_ctx* ctx, const float* features, int64_t n, float* scores) {
  if (!ctx || !features || !scores) return GS_EINVAL;
  ctx->err.clear();
  GS_HIP(ctx, hipSetDevice(ctx->device));
  return policy_predict(ctx, features, n, scores);
}

gs_status gs_policy_get_params(gs_ctx* ctx, float* params, int64_t n) {
  if (!ctx || !params) return GS_EINVAL;
  if (n != policy_param_floats()) GS_FAIL(ctx, GS_EINVAL, "the parameter array holds 5542 floats");
  if (!ctx->policy.ready) GS_FAIL(ctx, GS_EINVAL, "the learned policy has no parameters");
  policy_get_params(ctx->policy, params);
  return GS_OK;
}

gs_status gs_policy_set_params(gs_ctx* ctx, const float* params, int64_t n) {
  if (!ctx || !params) return GS_EINVAL;
  ctx->err.clear();
  if (n != policy_param_floats()) GS_FAIL(ctx, GS_EINVAL, "the parameter array holds 5542 floats");
  return policy_set_params(ctx, params);
}

gs_status gs_policy_save(gs_ctx* ctx, const char* path) {
  if (!ctx || !path) return GS_EINVAL;
  ctx->err.clear();
  return policy_save(ctx, path);
}

gs_status gs_policy_load(gs_ctx* ctx, const char* path) {
  if (!ctx || !path) return GS_EINVAL;
  ctx->err.clear();
  return policy_load(ctx, path);
}

gs_status gs_get_trace(gs_ctx* ctx, int64_t* n_records, int32_t* records) {
  if (!ctx || !n_records) return GS_EINVAL;
  *n_records = (int64_t)(ctx->trace.size() / 6);
  if (records) std::copy(ctx->trace.begin(), ctx->trace.end(), records);
  return GS_OK;
}

// Workload signature of the autotuner: method, policy, order limit and
// method mask, dimension, mono/bichromatic, M and N to a factor of 2^(1/2),
// the bandwidth count and range to a quarter decade, eps to an eighth decade.
static std::string autotune_key(const gs_options& o, int D, bool mono, int64_t M, int64_t N,
                                const std::vector<double>& hs, double eps) {
  double hmin = hs[0], hmax = hs[0];
  for (double h : hs) {
    hmin = std::min(hmin, h);
    hmax = std::max(hmax, h);
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%d/%d/%d/%d/%d/%d/%d/%d/%ld/%ld/%zu/%ld/%ld/%ld", o.method, o.policy,
                o.plimit, o.fmm_mask, o.node_bounds, o.pair_order, D, mono ? 1 : 0, std::lround(2.0 * std::log2((double)M)),
                std::lround(2.0 * std::log2((double)N)), hs.size(), std::lround(4.0 * std::log10(hmin)),
                std::lround(4.0 * std::log10(hmax)), std::lround(8.0 * std::log10(eps)));
  return buf;
}

gs_status gauss_sum(gs_ctx* ctx, const double* queries, int64_t M, const double* refs,
                    const double* weights, int64_t N, int32_t D, const double* bandwidths,
                    int32_t n_h, double eps, double* G_out, const gs_options* opt_in) {
  if (!ctx) return GS_EINVAL;
  ctx->err.clear();
  gs_options opt;
  gs_default_options(&opt);
  if (opt_in) {
    if (opt_in->struct_size != (int32_t)sizeof(gs_options))
      GS_FAIL(ctx, GS_EINVAL, "gs_options.struct_size does not match this library");
    opt = *opt_in;
  }
  if (!queries || !refs || !weights || !bandwidths || !G_out)
    GS_FAIL(ctx, GS_EINVAL, "null array pointer");
  if (M < 1 || N < 1 || n_h < 1) GS_FAIL(ctx, GS_EINVAL, "M, N and n_h must be >= 1");
  if (D < 1 || D > kMaxD) GS_FAIL(ctx, GS_EINVAL, "D must be in [1, 64]");
  if (M > INT32_MAX / 2 || N > INT32_MAX / 2) GS_FAIL(ctx, GS_EOVERFLOW, "M and N must be < 2^30");
  if (n_h > 4096) GS_FAIL(ctx, GS_EINVAL, "at most 4096 bandwidths per call");
  if (opt.method < GS_DUALTREE || opt.method > GS_DFTO) GS_FAIL(ctx, GS_EINVAL, "unknown method");
  if (opt.method == GS_DFTO && opt.node_bounds != GS_BOUNDS_BOX)
    GS_FAIL(ctx, GS_EINVAL, "GS_DFTO's bounds need node_bounds = GS_BOUNDS_BOX");
  if (opt.method == GS_DFTO && (opt.policy != GS_RULE || opt.log_pairs))
    GS_FAIL(ctx, GS_EINVAL, "the learned policy and its logging serve GS_DUALTREE only");
  if (opt.method != GS_EXHAUSTIVE && !(eps > 0.0 && eps < 1.0))
    GS_FAIL(ctx, GS_EINVAL, "eps must be in (0, 1)");
  if (opt.leaf_size < 1 || opt.leaf_size > 1024) GS_FAIL(ctx, GS_EINVAL, "leaf_size must be in [1, 1024]");
  if (opt.h_chunk < 0) GS_FAIL(ctx, GS_EINVAL, "h_chunk must be >= 0");
  if (opt.kernel_timing < 0 || opt.kernel_timing > 2) GS_FAIL(ctx, GS_EINVAL, "kernel_timing must be 0, 1 or 2");
  if (opt.node_bounds != GS_BOUNDS_BOX && opt.node_bounds != GS_BOUNDS_SPHERE_RECT)
    GS_FAIL(ctx, GS_EINVAL, "node_bounds must be GS_BOUNDS_BOX or GS_BOUNDS_SPHERE_RECT");
  if (opt.max_frontier < 0) GS_FAIL(ctx, GS_EINVAL, "max_frontier must be >= 0");
  if (opt.pair_order != GS_ORDER_TREE && opt.pair_order != GS_ORDER_FAR_FIRST)
    GS_FAIL(ctx, GS_EINVAL, "pair_order must be GS_ORDER_TREE or GS_ORDER_FAR_FIRST");
  if (opt.debug_fail_alloc < 0) GS_FAIL(ctx, GS_EINVAL, "debug_fail_alloc must be >= 0");
  if (!(opt.eps_round_share >= 0.0 && opt.eps_round_share < 1.0))
    GS_FAIL(ctx, GS_EINVAL, "eps_round_share must be in [0, 1)");
  if (opt.policy != GS_RULE && opt.policy != GS_LEARNED) GS_FAIL(ctx, GS_EINVAL, "unknown policy");
  if (opt.policy == GS_LEARNED && !ctx->policy.ready)
    GS_FAIL(ctx, GS_EINVAL, "policy = GS_LEARNED needs parameters: train or load the policy first");
  if (!(opt.log_explore >= 0.0 && opt.log_explore <= 1.0))
    GS_FAIL(ctx, GS_EINVAL, "log_explore must be in [0, 1]");
  if (opt.log_pairs && opt.policy == GS_LEARNED)
    GS_FAIL(ctx, GS_EINVAL, "log_pairs records the rule's decisions: use policy = GS_RULE");
  if (opt.log_pairs) {
    opt.keep_trace = 1;     // the records are built from the trace,
    opt.kernel_timing = 1;  // with costs measured in this call
  }
  GS_HIP(ctx, hipSetDevice(ctx->device));
  const double t_start = now_ms();
  hipStream_t st = ctx->stream;
  AllocFaultScope fault_scope(ctx, opt.debug_fail_alloc);
  DrainOnFailure drain{ctx};

  // Bandwidths on the host.
  std::vector<double> hs(n_h);
  if (is_device_pointer(bandwidths)) {
    hipError_t pe = hipSuccess;
    auto* ph = static_cast<double*>(ctx->ws.get_pinned("hs_read", n_h * sizeof(double), &pe));
    if (!ph) GS_FAIL(ctx, GS_ENOMEM, "pinned host allocation failed");
    GS_HIP(ctx, hipMemcpyAsync(ph, bandwidths, n_h * sizeof(double), hipMemcpyDeviceToHost, st));
    GS_HIP(ctx, hipStreamSynchronize(st));
    std::copy(ph, ph + n_h, hs.begin());
  } else {
    std::copy(bandwidths, bandwidths + n_h, hs.begin());
  }
  for (double h : hs)
    if (!(h > 0.0) || !std::isfinite(h)) GS_FAIL(ctx, GS_EINVAL, "every bandwidth must be finite and > 0");

  const bool mono = opt.monochromatic == 1 || (opt.monochromatic == -1 && queries == refs && M == N);
  if (mono && M != N) GS_FAIL(ctx, GS_EINVAL, "monochromatic requires M == N");

  // Stage inputs on the device (validated, -0.0 canonicalised).
  int* bad = WS(int, "bad_flag", 1);
  GS_HIP(ctx, hipMemsetAsync(bad, 0, sizeof(int), st));
  auto stage = [&](const double* src, int64_t n, const char* raw_name, const char* soa_name,
                   const char* aos_name, double** soa, double** aos) -> gs_status {
    const double* dsrc = src;
    if (!is_device_pointer(src)) {
      double* raw = WS(double, raw_name, n * D);
      GS_HIP(ctx, hipMemcpyAsync(raw, src, n * D * sizeof(double), hipMemcpyHostToDevice, st));
      dsrc = raw;
    }
    *soa = WS(double, soa_name, n * D);
    *aos = WS(double, aos_name, n * D);
    GS_HIP(ctx, launch_stage_points(dsrc, n, D, *soa, *aos, bad, st));
    return GS_OK;
  };
  DeviceInputs in;
  in.M = M;
  in.N = N;
  in.D = D;
  in.mono = mono;
  gs_status s = stage(refs, N, "raw_r", "r_soa", "r_aos", &in.r_soa, &in.r_aos);
  if (s != GS_OK) return s;
  if (mono) {
    in.q_soa = in.r_soa;
    in.q_aos = in.r_aos;
  } else {
    s = stage(queries, M, "raw_q", "q_soa", "q_aos", &in.q_soa, &in.q_aos);
    if (s != GS_OK) return s;
  }
  in.w = WS(double, "w", N);
  if (is_device_pointer(weights))
    GS_HIP(ctx, hipMemcpyAsync(in.w, weights, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  else
    GS_HIP(ctx, hipMemcpyAsync(in.w, weights, N * sizeof(double), hipMemcpyHostToDevice, st));
  GS_HIP(ctx, launch_check_positive(in.w, N, bad, st));
  int bad_h = 0;
  {
    hipError_t pe = hipSuccess;
    auto* pb = static_cast<int*>(ctx->ws.get_pinned("bad_read", sizeof(int), &pe));
    if (!pb) GS_FAIL(ctx, GS_ENOMEM, "pinned host allocation failed");
    GS_HIP(ctx, hipMemcpyAsync(pb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    GS_HIP(ctx, hipStreamSynchronize(st));
    bad_h = *pb;
  }
  if (bad_h & 1) GS_FAIL(ctx, GS_EINVAL, "a coordinate is NaN or infinite");
  if (bad_h & 2) GS_FAIL(ctx, GS_EINVAL, "every weight must be finite and > 0");
  const double t_staged = now_ms();

  // Output buffer.
  const bool out_dev = is_device_pointer(G_out);
  double* Gd = out_dev ? G_out : WS(double, "G_tmp", (int64_t)n_h * M);

  // One summation with the options o into Gd; resets the statistics.
  auto run_once = [&](const gs_options& o) -> gs_status {
    GS_HIP(ctx, hipStreamSynchronize(st));
    ctx->stats_pending = nullptr;
    flush_kernel_timers(ctx);  // timers of an earlier trial
    std::memset(&ctx->stats, 0, sizeof(ctx->stats));
    ctx->stats.struct_size = sizeof(gs_stats);
    ctx->stats.n_h = n_h;
    ctx->stats.t_stage_ms = t_staged - t_start;
    ctx->pair_counts.assign((size_t)n_h * 6, 0);
    ctx->trace.clear();
    ctx->trace_feat.clear();
    ctx->trace_feas.clear();
    ctx->policy.log.clear();
    ctx->policy.log_keys.clear();
    ctx->host_tree[0].valid = ctx->host_tree[1].valid = false;
    ctx->kernel_timing = o.kernel_timing != 0;
    ctx->timing_mask = o.kernel_timing == 1   ? ~0u
                       : o.kernel_timing == 2 ? (1u << GS_K_BASE) | (1u << GS_K_EXHAUSTIVE)
                                              : 0u;
    if (o.method == GS_EXHAUSTIVE) {
      float* rec = WS(float, "ex_rec", N * exhaustive_record_stride(D));
      unsigned long long* wb = WS(unsigned long long, "wmax_bits", 1);
      GS_HIP(ctx, launch_exhaustive_records(in.r_aos, in.w, N, D, rec, wb, st));
      double* partial = WS(double, "ex_partial", exhaustive_partial_elems(M, N, n_h));
      KernelTimer kt(ctx, ctx->kernel_timing, GS_K_EXHAUSTIVE, st);
      GS_HIP(ctx, launch_exhaustive(in.q_aos, M, rec, N, D, hs.data(), n_h, wb, partial, Gd, st));
      kt.stop(st, 1);
      return GS_OK;
    }
    return run_dualtree(ctx, in, hs, eps, o, Gd);
  };

  // Autotuning (dual-tree methods): the fastest of the leaf sizes 32..256 and,
  // for GS_DUALTREE, the exhaustive path, per workload signature, measured
  // once per context and reused.
  int trials = 0;
  if (opt.autotune && opt.method != GS_EXHAUSTIVE && !opt.keep_trace) {
    const std::string key = autotune_key(opt, D, mono, M, N, hs, eps);
    auto it = ctx->tuned.find(key);
    if (it == ctx->tuned.end()) {
      std::vector<std::pair<int, int>> cand;  // (method, leaf)
      for (int leaf : {32, 64, 128, 256}) cand.push_back({opt.method, leaf});
      if (opt.method == GS_DUALTREE) cand.push_back({GS_EXHAUSTIVE, opt.leaf_size});
      double best_ms = 0.0;
      std::pair<int, int> best = cand[0];
      for (const auto& c : cand) {
        gs_options o = opt;
        o.method = c.first;
        o.leaf_size = c.second;
        o.kernel_timing = 0;
        // The exhaustive path runs at most ~5e12 pair-evaluations/s on one
        // MI355X: skip it when even that rate loses to the best leaf size.
        if (c.first == GS_EXHAUSTIVE && best_ms > 0.0 && (double)M * (double)N * n_h / 5e9 > best_ms) continue;
        double ms = 0.0;
        for (int rep = 0; rep < 2; ++rep) {  // the first run also sizes the workspace
          const double t0 = now_ms();
          s = run_once(o);
          if (s != GS_OK) return s;
          GS_HIP(ctx, hipStreamSynchronize(st));
          ms = now_ms() - t0;
          ++trials;
          if (ms > 100.0) break;  // allocation no longer matters at this size
        }
        if (best_ms == 0.0 || ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
      it = ctx->tuned.emplace(key, best).first;
    }
    opt.method = it->second.first;
    opt.leaf_size = it->second.second;
  }
  s = run_once(opt);
  if (s != GS_OK) return s;
  ctx->stats.autotune_trials = trials;
  ctx->stats.tuned_method = opt.method;
  ctx->stats.tuned_leaf_size = opt.leaf_size;
  if (!out_dev) {
    GS_HIP(ctx, hipMemcpyAsync(G_out, Gd, (size_t)n_h * M * sizeof(double), hipMemcpyDeviceToHost, st));
    GS_HIP(ctx, hipStreamSynchronize(st));
  } else if (opt.blocking) {
    GS_HIP(ctx, hipStreamSynchronize(st));
  }
  if (!out_dev || opt.blocking) {
    finish_dualtree_stats(ctx);
    flush_kernel_timers(ctx);
  }
  ctx->stats.t_total_ms = now_ms() - t_start;
  ctx->stats.pair_evals_per_s = (double)M * (double)N * (double)n_h / (ctx->stats.t_total_ms * 1e-3);
  ctx->stats.workspace_requests = ctx->alloc_requests;
  if (opt.log_pairs && opt.log_path) {
    s = policy_write_log(ctx, opt.log_path);
    if (s != GS_OK) return s;
  }
  drain.ok = true;
  return GS_OK;
}

gs_status gs_lscv(gs_ctx* ctx, const double* points, int64_t N, int32_t D, const double* bandwidths,
                  int32_t n_h, double eps, double* scores, double* bounds, const gs_options* opt_in) {
  if (!ctx) return GS_EINVAL;
  ctx->err.clear();
  if (!points || !bandwidths || !scores) GS_FAIL(ctx, GS_EINVAL, "null array pointer");
  if (N < 2) GS_FAIL(ctx, GS_EINVAL, "the score needs N >= 2 points");
  if (n_h < 1 || n_h > 2048) GS_FAIL(ctx, GS_EINVAL, "n_h must be in [1, 2048]");
  gs_options opt;
  gs_default_options(&opt);
  if (opt_in) {
    if (opt_in->struct_size != (int32_t)sizeof(gs_options))
      GS_FAIL(ctx, GS_EINVAL, "gs_options.struct_size does not match this library");
    opt = *opt_in;
  }
  if (opt.keep_trace || opt.log_pairs) GS_FAIL(ctx, GS_EINVAL, "keep_trace and log_pairs do not apply to gs_lscv");
  opt.monochromatic = 1;
  if (opt.debug_fail_alloc < 0) GS_FAIL(ctx, GS_EINVAL, "debug_fail_alloc must be >= 0");
  GS_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  AllocFaultScope fault_scope(ctx, opt.debug_fail_alloc);
  DrainOnFailure drain{ctx};
  std::vector<double> hs(n_h);
  if (is_device_pointer(bandwidths)) {
    GS_HIP(ctx, hipMemcpyAsync(hs.data(), bandwidths, n_h * sizeof(double), hipMemcpyDeviceToHost, st));
    GS_HIP(ctx, hipStreamSynchronize(st));
  } else {
    std::copy(bandwidths, bandwidths + n_h, hs.begin());
  }
  for (double h : hs)
    if (!(h > 0.0) || !std::isfinite(h)) GS_FAIL(ctx, GS_EINVAL, "every bandwidth must be finite and > 0");
  // one sweep over h and sqrt(2) h, unit weights, the points against themselves
  std::vector<double> ext(2 * (size_t)n_h);
  for (int k = 0; k < n_h; ++k) {
    ext[k] = hs[k];
    ext[n_h + k] = std::sqrt(2.0) * hs[k];
  }
  double* w = WS(double, "lscv_w", N);
  GS_HIP(ctx, launch_fill(w, N, 1.0, st));
  double* G = WS(double, "lscv_G", 2 * (int64_t)n_h * N);
  gs_status s = gauss_sum(ctx, points, N, points, w, N, D, ext.data(), 2 * n_h, eps, G, &opt);
  if (s != GS_OK) return s;
  double* sums = WS(double, "lscv_sums", 2 * n_h);
  double* dh = WS(double, "lscv_hs", n_h);
  double* out = WS(double, "lscv_out", 2 * n_h);
  GS_HIP(ctx, hipMemcpyAsync(dh, hs.data(), n_h * sizeof(double), hipMemcpyHostToDevice, st));
  GS_HIP(ctx, launch_lscv_reduce(G, 2 * n_h, N, sums, st));
  // the exhaustive path's float tiles stay within 1e-3 relative per query
  const double e = opt.method == GS_EXHAUSTIVE ? 1e-3 : eps;
  GS_HIP(ctx, launch_lscv_combine(sums, dh, n_h, N, D, e, out, out + n_h, st));
  GS_HIP(ctx, hipMemcpyAsync(scores, out, n_h * sizeof(double), hipMemcpyDefault, st));
  if (bounds) GS_HIP(ctx, hipMemcpyAsync(bounds, out + n_h, n_h * sizeof(double), hipMemcpyDefault, st));
  GS_HIP(ctx, hipStreamSynchronize(st));
  ctx->stats.workspace_requests = ctx->alloc_requests;
  drain.ok = true;
  return GS_OK;
}

}  // extern "C"
