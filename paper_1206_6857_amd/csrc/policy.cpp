// Host side of the learned pair policy: parameters and standardisation,
// training records from a decision trace, training, prediction, files.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "gs_host.h"
#include "gs_policy.h"

namespace gs {

namespace {

constexpr int oW1 = 0;
constexpr int ob1 = oW1 + kPolicyHidden * kPolicyIn;
constexpr int oW2 = ob1 + kPolicyHidden;
constexpr int ob2 = oW2 + kPolicyHidden * kPolicyHidden;
constexpr int oW3 = ob2 + kPolicyHidden;
constexpr int ob3 = oW3 + kPolicyOut * kPolicyHidden;

const char kParamMagic[8] = {'G', 'S', 'P', 'O', 'L', 'I', 'C', 'Y'};
const char kLogMagic[8] = {'G', 'S', 'P', 'O', 'L', 'L', 'O', 'G'};

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * 0x1.0p-53; }

uint64_t binom_u(int n, int k) {
  if (k < 0 || k > n) return 0;
  if (k > n - k) k = n - k;
  uint64_t c = 1;
  for (int i = 1; i <= k; ++i) c = c * (uint64_t)(n - k + i) / (uint64_t)i;
  return c;
}

#define P_HIP(call)                                                                   \
  do {                                                                                \
    hipError_t _e = (call);                                                           \
    if (_e != hipSuccess) {                                                           \
      (void)hipGetLastError();                                                        \
      ctx->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(_e); \
      return _e == hipErrorOutOfMemory ? GS_ENOMEM : GS_EDEVICE;                      \
    }                                                                                 \
  } while (0)

#define P_FAIL(code, msg) \
  do {                    \
    ctx->err = (msg);     \
    return (code);        \
  } while (0)

template <class T>
T* wsbuf(gs_ctx_base* ctx, const char* name, size_t count, gs_status* st) {
  hipError_t e = hipSuccess;
  void* p = ctx->ws.get(name, std::max<size_t>(count, 1) * sizeof(T), ctx, &e);
  if (!p) {
    ctx->err = std::string("device allocation failed for '") + name + "'";
    *st = GS_ENOMEM;
  }
  return static_cast<T*>(p);
}

#define WSBUF(T, name, count)                                  \
  ({                                                           \
    gs_status _st = GS_OK;                                     \
    T* _p = wsbuf<T>(ctx, name, (size_t)(count), &_st);        \
    if (!_p) return _st;                                       \
    _p;                                                        \
  })

PolicyNorm norm_of(const PolicyState& ps) {
  PolicyNorm nm;
  for (int k = 0; k < kPolicyIn; ++k) {
    nm.mu_x[k] = ps.mu_x[k];
    nm.isd_x[k] = 1.0f / ps.sd_x[k];
  }
  nm.mu_y = ps.mu_y;
  nm.isd_y = 1.0f / ps.sd_y;
  return nm;
}

// A-operand tiles of the three weight matrices (see k_policy.hip).
std::vector<_Float16> pack_weights(const std::vector<float>& th) {
  std::vector<_Float16> w((size_t)kPolicyTiles * 64 * 4);
  for (int t = 0; t < kPolicyTiles; ++t)
    for (int l = 0; l < 64; ++l)
      for (int e = 0; e < 4; ++e) {
        const int i = l % 16, k = 4 * (l / 16) + e;
        float v = 0.0f;
        if (t < 4) {
          v = th[oW1 + (16 * t + i) * kPolicyIn + k];
        } else if (t < 20) {
          const int r = (t - 4) / 4, kt = (t - 4) % 4;
          v = th[oW2 + (16 * r + i) * kPolicyHidden + 16 * kt + k];
        } else if (i < kPolicyOut) {
          v = th[oW3 + i * kPolicyHidden + 16 * (t - 20) + k];
        }
        w[((size_t)t * 64 + l) * 4 + e] = (_Float16)v;
      }
  return w;
}

// Records must be readable by the device: copy host records into the workspace.
gs_status stage_records(gs_ctx_base* ctx, const float* rec, int64_t n, const char* name, const float** out) {
  if (is_device_pointer(rec)) {
    *out = rec;
    return GS_OK;
  }
  float* d = WSBUF(float, name, (size_t)n * kPolicyRecord);
  P_HIP(hipMemcpyAsync(d, rec, sizeof(float) * n * kPolicyRecord, hipMemcpyHostToDevice, ctx->stream));
  *out = d;
  return GS_OK;
}

}  // namespace

void policy_default_costs(PolicyState& ps) {
  // Measured on one MI355X (D=3, 100k points, 10 bandwidths, leaf 128): the
  // kernel time of each work type over one sweep with the rule divided by its
  // units (c_h2l: the H2L kernel's per-term work equals DH's).  A logged call
  // (log_pairs) replaces the work-type costs by its own measurements.
  ps.c_pair = 0.9;
  ps.c_dh = 3.0e-4;
  ps.c_dl = 3.9e-3;
  ps.c_h2l = 3.0e-4;
  ps.c_base = 2.65e-4;
}

gs_status policy_device_model(gs_ctx_base* ctx, PolicyDevModel* m) {
  PolicyState& ps = ctx->policy;
  if (!ps.ready) P_FAIL(GS_EINVAL, "the learned policy has no parameters: train or load it first");
  float* dth = WSBUF(float, "pol_theta", 3 * kPolicyParams);
  _Float16* dw = WSBUF(_Float16, "pol_wpack", kPolicyTiles * 64 * 4);
  if (!ps.dev_fresh) {
    const std::vector<_Float16> w = pack_weights(ps.theta);
    P_HIP(hipMemcpyAsync(dth, ps.theta.data(), sizeof(float) * kPolicyParams, hipMemcpyHostToDevice,
                         ctx->stream));
    P_HIP(hipMemcpyAsync(dw, w.data(), sizeof(_Float16) * w.size(), hipMemcpyHostToDevice, ctx->stream));
    P_HIP(hipStreamSynchronize(ctx->stream));
    ps.dev_fresh = true;
  }
  m->wpack = dw;
  m->b1 = dth + ob1;
  m->b2 = dth + ob2;
  m->b3 = dth + ob3;
  for (int k = 0; k < kPolicyIn; ++k) {
    m->mu_x[k] = ps.mu_x[k];
    m->isd_x[k] = 1.0f / ps.sd_x[k];
  }
  return GS_OK;
}

// Measured cost model: each work type's unit cost becomes this call's kernel
// time of the type divided by its units (from the trace), where the type's
// kernels ran long enough (>= 0.05 ms) for launch latency not to dominate;
// the other unit costs are kept.  The cost of deciding a pair is not taken
// from a logged call: logging computes every pair's features and admitted
// orders, which a call that only decides does not.
void policy_calibrate_costs(gs_ctx_base* ctx, int D) {
  PolicyState& ps = ctx->policy;
  const HostTree& rt = ctx->host_tree[0];
  const HostTree& qt = ctx->host_tree[1];
  const std::vector<int32_t>& tr = ctx->trace;
  const int64_t n = (int64_t)tr.size() / 6;
  if (ps.costs_pinned || n == 0 || !qt.valid || !rt.valid) return;
  double u[5] = {(double)n, 0.0, 0.0, 0.0, 0.0};  // pairs, DH, DL, H2L, base
  for (int64_t i = 0; i < n; ++i) {
    const int code = tr[6 * i + 4], p = tr[6 * i + 5];
    const double NQ = qt.count[tr[6 * i + 2]], NR = rt.count[tr[6 * i + 3]];
    const double C = p > 0 ? (double)binom_u(D + p - 1, D) : 0.0;
    if (code == 1) u[1] += NQ * C;
    else if (code == 2) u[2] += NR * C;
    else if (code == 3) u[3] += C * C;
    else if (code == 4) u[4] += NQ * NR;
  }
  const gs_stats& S = ctx->stats;
  const double ms[5] = {S.k_ms[GS_K_DECIDE], S.k_ms[GS_K_DH], S.k_ms[GS_K_DL], S.k_ms[GS_K_H2L], S.k_ms[GS_K_BASE]};
  double* c[5] = {&ps.c_pair, &ps.c_dh, &ps.c_dl, &ps.c_h2l, &ps.c_base};
  for (int k = 1; k < 5; ++k)
    if (u[k] > 0.0 && ms[k] >= 0.05) *c[k] = ms[k] * 1e6 / u[k];
}

// Records of the last logged traversal, from ctx->trace and the per-row
// features and admitted orders.  Cost of a decided pair (ns): c_pair, plus
// N_Q C(D+p-1,D) c_dh (DH), N_R C c_dl (DL), C^2 c_h2l (H2L), N_Q N_R c_base
// (base case), or the children's cost-to-go (split).
gs_status policy_build_records(gs_ctx_base* ctx, int D, const std::vector<double>& hs) {
  PolicyState& ps = ctx->policy;
  const HostTree& rt = ctx->host_tree[0];
  const HostTree& qt = ctx->host_tree[1];
  const std::vector<int32_t>& tr = ctx->trace;
  const int64_t n = (int64_t)tr.size() / 6;
  if ((int64_t)ctx->trace_feat.size() != n * kPolicyIn || (int64_t)ctx->trace_feas.size() != n)
    P_FAIL(GS_EINTERNAL, "policy log: trace and features out of step");
  if (qt.n_nodes >= (1 << 26) || rt.n_nodes >= (1 << 26) || hs.size() >= 4096)
    P_FAIL(GS_EOVERFLOW, "policy log: trees or bandwidth list too large to key");
  auto key = [](int64_t h, int64_t Q, int64_t R) {
    return ((uint64_t)h << 52) | ((uint64_t)Q << 26) | (uint64_t)R;
  };
  std::unordered_map<uint64_t, int64_t> index;
  index.reserve((size_t)n * 2);
  int max_level = 0;
  for (int64_t i = 0; i < n; ++i) {
    index[key(tr[6 * i], tr[6 * i + 2], tr[6 * i + 3])] = i;
    max_level = std::max(max_level, (int)tr[6 * i + 1]);
  }
  std::vector<std::vector<int64_t>> by_level(max_level + 1);
  for (int64_t i = 0; i < n; ++i) by_level[tr[6 * i + 1]].push_back(i);
  auto terms = [&](int p) { return (double)binom_u(D + p - 1, D); };
  auto action = [&](int code, int p, double NQ, double NR) {
    double c = ps.c_pair;
    if (code == 1) c += NQ * terms(p) * ps.c_dh;
    else if (code == 2) c += NR * terms(p) * ps.c_dl;
    else if (code == 3) c += terms(p) * terms(p) * ps.c_h2l;
    else if (code == 4) c += NQ * NR * ps.c_base;
    return c;
  };
  std::vector<double> ctg((size_t)n, 0.0);
  for (int lev = max_level; lev >= 0; --lev) {
    for (int64_t i : by_level[lev]) {
      const int h = tr[6 * i], Q = tr[6 * i + 2], R = tr[6 * i + 3], code = tr[6 * i + 4], p = tr[6 * i + 5];
      double c = action(code, p, (double)qt.count[Q], (double)rt.count[R]);
      if (code == 5) {
        const int qn = qt.left[Q] < 0 ? 1 : 2, rn = rt.left[R] < 0 ? 1 : 2;
        for (int a = 0; a < qn; ++a)
          for (int b = 0; b < rn; ++b) {
            const int qc = qn == 1 ? Q : qt.left[Q] + a;
            const int rc = rn == 1 ? R : rt.left[R] + b;
            auto it = index.find(key(h, qc, rc));
            if (it == index.end()) P_FAIL(GS_EINTERNAL, "policy log: a split pair has no child in the trace");
            c += ctg[it->second];
          }
      }
      ctg[i] = c;
    }
  }
  ps.log.clear();
  ps.log_keys.clear();
  for (int64_t i = 0; i < n; ++i) {
    const int f = ctx->trace_feas[i];
    if (!(f & 0x8000)) continue;
    const int Q = tr[6 * i + 2], R = tr[6 * i + 3], code = tr[6 * i + 4];
    const double NQ = qt.count[Q], NR = rt.count[R];
    float rec[kPolicyRecord];
    for (int k = 0; k < kPolicyIn; ++k) rec[k] = ctx->trace_feat[i * kPolicyIn + k];
    const int q[3] = {f & 15, (f >> 4) & 15, (f >> 8) & 15};
    for (int k = 0; k < 3; ++k) {
      rec[kPolicyIn + k] = q[k] ? (float)std::log2(action(k + 1, q[k], NQ, NR)) : 0.0f;
      rec[kPolicyIn + kPolicyOut + k] = q[k] ? 1.0f : 0.0f;
    }
    const bool direct = code == 4 || code == 5;
    rec[kPolicyIn + 3] = direct ? (float)std::log2(ctg[i]) : 0.0f;
    rec[kPolicyIn + kPolicyOut + 3] = direct ? 1.0f : 0.0f;
    ps.log.insert(ps.log.end(), rec, rec + kPolicyRecord);
    const int32_t k4[4] = {tr[6 * i], tr[6 * i + 1], Q, R};
    ps.log_keys.insert(ps.log_keys.end(), k4, k4 + 4);
  }
  return GS_OK;
}

gs_status policy_train(gs_ctx_base* ctx, const float* rec_in, int64_t n, const gs_train_opts& o,
                       float* final_loss) {
  PolicyState& ps = ctx->policy;
  hipStream_t st = ctx->stream;
  if (n < 1 || n > INT32_MAX / 2) P_FAIL(GS_EINVAL, "policy training needs 1 .. 2^30 records");
  if (o.steps < 0 || o.batch < 1 || !(o.lr > 0.0)) P_FAIL(GS_EINVAL, "bad training options");
  // host copy for the standardisation
  std::vector<float> host;
  const float* rec_h = rec_in;
  if (is_device_pointer(rec_in)) {
    host.resize((size_t)n * kPolicyRecord);
    P_HIP(hipMemcpy(host.data(), rec_in, sizeof(float) * host.size(), hipMemcpyDeviceToHost));
    rec_h = host.data();
  }
  if (o.reinit || !ps.ready) {
    for (int k = 0; k < kPolicyIn; ++k) {
      double s = 0.0, s2 = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        const double v = rec_h[i * kPolicyRecord + k];
        s += v;
        s2 += v * v;
      }
      const double mu = s / (double)n;
      const double var = std::max(0.0, s2 / (double)n - mu * mu);
      ps.mu_x[k] = (float)mu;
      ps.sd_x[k] = var > 1e-12 ? (float)std::sqrt(var) : 1.0f;
    }
    double s = 0.0, s2 = 0.0, cnt = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < kPolicyOut; ++k)
        if (rec_h[i * kPolicyRecord + kPolicyIn + kPolicyOut + k] != 0.0f) {
          const double v = rec_h[i * kPolicyRecord + kPolicyIn + k];
          s += v;
          s2 += v * v;
          cnt += 1.0;
        }
    const double mu = cnt > 0.0 ? s / cnt : 0.0;
    const double var = cnt > 0.0 ? std::max(0.0, s2 / cnt - mu * mu) : 1.0;
    ps.mu_y = (float)mu;
    ps.sd_y = var > 1e-12 ? (float)std::sqrt(var) : 1.0f;
    // He-uniform weights, zero biases
    uint64_t seed = o.seed;
    ps.theta.assign(kPolicyParams, 0.0f);
    auto fill = [&](int off, int count, int fan_in) {
      const double a = std::sqrt(6.0 / fan_in);
      for (int i = 0; i < count; ++i) ps.theta[off + i] = (float)((2.0 * uniform01(seed) - 1.0) * a);
    };
    fill(oW1, kPolicyHidden * kPolicyIn, kPolicyIn);
    fill(oW2, kPolicyHidden * kPolicyHidden, kPolicyHidden);
    fill(oW3, kPolicyOut * kPolicyHidden, kPolicyHidden);
    ps.ready = true;
  }
  const float* rec = nullptr;
  gs_status s0 = stage_records(ctx, rec_in, n, "pol_rec", &rec);
  if (s0 != GS_OK) return s0;
  float* dth = WSBUF(float, "pol_theta", 3 * kPolicyParams);
  int32_t* didx = WSBUF(int32_t, "pol_idx", n);
  const int B = (int)std::min<int64_t>(o.batch, n);
  const int nw = policy_grad_waves(B);
  const int nw_all = policy_grad_waves((int)n);
  float* partial = WSBUF(float, "pol_partial", (size_t)std::max(nw, nw_all) * (kPolicyParams + 2));
  float* dstats = WSBUF(float, "pol_stats", 2);
  P_HIP(hipMemcpyAsync(dth, ps.theta.data(), sizeof(float) * kPolicyParams, hipMemcpyHostToDevice, st));
  P_HIP(hipMemsetAsync(dth + kPolicyParams, 0, sizeof(float) * 2 * kPolicyParams, st));
  const PolicyNorm nm = norm_of(ps);
  std::vector<int32_t> perm((size_t)n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  uint64_t rs = o.seed ^ 0x5deece66dull;
  int64_t cursor = n;  // forces a shuffle before the first step
  PolicyAdam ad;
  ad.lr = (float)o.lr;
  double b1p = 1.0, b2p = 1.0;
  for (int step = 1; step <= o.steps; ++step) {
    if (cursor + B > n) {
      for (int64_t i = n - 1; i > 0; --i) {
        const int64_t j = (int64_t)(splitmix64(rs) % (uint64_t)(i + 1));
        std::swap(perm[i], perm[j]);
      }
      P_HIP(hipMemcpyAsync(didx, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
      P_HIP(hipStreamSynchronize(st));
      cursor = 0;
    }
    b1p *= ad.beta1;
    b2p *= ad.beta2;
    ad.bc1 = (float)(1.0 - b1p);
    ad.bc2 = (float)(1.0 - b2p);
    P_HIP(launch_policy_grad(rec, didx + cursor, B, dth, nm, partial, nw, nullptr, dth, dth + kPolicyParams,
                             dth + 2 * kPolicyParams, ad, dstats, st));
    cursor += B;
  }
  // loss over all records at the final parameters
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  P_HIP(hipMemcpyAsync(didx, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  P_HIP(launch_policy_grad(rec, didx, (int)n, dth, nm, partial, nw_all, nullptr, nullptr, nullptr, nullptr, ad,
                           dstats, st));
  float stats[2] = {0.0f, 0.0f};
  P_HIP(hipMemcpyAsync(stats, dstats, sizeof(stats), hipMemcpyDeviceToHost, st));
  P_HIP(hipMemcpyAsync(ps.theta.data(), dth, sizeof(float) * kPolicyParams, hipMemcpyDeviceToHost, st));
  P_HIP(hipStreamSynchronize(st));
  ps.dev_fresh = false;
  if (final_loss) *final_loss = stats[0];
  return GS_OK;
}

gs_status policy_gradient(gs_ctx_base* ctx, const float* rec_in, int64_t n, float* grad, float* loss) {
  PolicyState& ps = ctx->policy;
  hipStream_t st = ctx->stream;
  if (!ps.ready) P_FAIL(GS_EINVAL, "the learned policy has no parameters: train or load it first");
  if (n < 1 || n > INT32_MAX / 2) P_FAIL(GS_EINVAL, "gradient needs 1 .. 2^30 records");
  const float* rec = nullptr;
  gs_status s0 = stage_records(ctx, rec_in, n, "pol_rec", &rec);
  if (s0 != GS_OK) return s0;
  float* dth = WSBUF(float, "pol_theta", 3 * kPolicyParams);
  float* dgrad = WSBUF(float, "pol_grad", kPolicyParams);
  int32_t* didx = WSBUF(int32_t, "pol_idx", n);
  const int nw = policy_grad_waves((int)n);
  float* partial = WSBUF(float, "pol_partial", (size_t)nw * (kPolicyParams + 2));
  float* dstats = WSBUF(float, "pol_stats", 2);
  std::vector<int32_t> id((size_t)n);
  for (int64_t i = 0; i < n; ++i) id[i] = (int32_t)i;
  P_HIP(hipMemcpyAsync(didx, id.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  P_HIP(hipMemcpyAsync(dth, ps.theta.data(), sizeof(float) * kPolicyParams, hipMemcpyHostToDevice, st));
  ps.dev_fresh = false;
  PolicyAdam ad;
  P_HIP(launch_policy_grad(rec, didx, (int)n, dth, norm_of(ps), partial, nw, dgrad, nullptr, nullptr, nullptr,
                           ad, dstats, st));
  float stats[2] = {0.0f, 0.0f};
  P_HIP(hipMemcpyAsync(stats, dstats, sizeof(stats), hipMemcpyDeviceToHost, st));
  if (grad) P_HIP(hipMemcpyAsync(grad, dgrad, sizeof(float) * kPolicyParams, hipMemcpyDefault, st));
  P_HIP(hipStreamSynchronize(st));
  if (loss) *loss = stats[0];
  return GS_OK;
}

gs_status policy_predict(gs_ctx_base* ctx, const float* feat_in, int64_t n, float* scores_out) {
  hipStream_t st = ctx->stream;
  if (n < 1 || n > INT32_MAX / 2) P_FAIL(GS_EINVAL, "prediction needs 1 .. 2^30 feature rows");
  PolicyDevModel m;
  gs_status s0 = policy_device_model(ctx, &m);
  if (s0 != GS_OK) return s0;
  const float* feat = feat_in;
  if (!is_device_pointer(feat_in)) {
    float* d = WSBUF(float, "pol_feat_in", (size_t)n * kPolicyIn);
    P_HIP(hipMemcpyAsync(d, feat_in, sizeof(float) * n * kPolicyIn, hipMemcpyHostToDevice, st));
    feat = d;
  }
  float4* out = WSBUF(float4, "pol_scores_out", n);
  P_HIP(launch_policy_infer_features((int)n, feat, m, out, st));
  P_HIP(hipMemcpyAsync(scores_out, out, sizeof(float4) * n, hipMemcpyDefault, st));
  P_HIP(hipStreamSynchronize(st));
  return GS_OK;
}

int64_t policy_param_floats() { return kPolicyParams + kPolicyNormFloats; }

void policy_get_params(const PolicyState& ps, float* out) {
  std::copy(ps.theta.begin(), ps.theta.end(), out);
  float* o = out + kPolicyParams;
  for (int k = 0; k < kPolicyIn; ++k) o[k] = ps.mu_x[k];
  for (int k = 0; k < kPolicyIn; ++k) o[kPolicyIn + k] = ps.sd_x[k];
  o[2 * kPolicyIn] = ps.mu_y;
  o[2 * kPolicyIn + 1] = ps.sd_y;
}

gs_status policy_set_params(gs_ctx_base* ctx, const float* in) {
  PolicyState& ps = ctx->policy;
  for (int i = 0; i < policy_param_floats(); ++i)
    if (!std::isfinite(in[i])) P_FAIL(GS_EINVAL, "policy parameters must be finite");
  const float* o = in + kPolicyParams;
  for (int k = 0; k < kPolicyIn; ++k)
    if (!(o[kPolicyIn + k] > 0.0f)) P_FAIL(GS_EINVAL, "policy standard deviations must be > 0");
  if (!(o[2 * kPolicyIn + 1] > 0.0f)) P_FAIL(GS_EINVAL, "policy standard deviations must be > 0");
  ps.theta.assign(in, in + kPolicyParams);
  for (int k = 0; k < kPolicyIn; ++k) {
    ps.mu_x[k] = o[k];
    ps.sd_x[k] = o[kPolicyIn + k];
  }
  ps.mu_y = o[2 * kPolicyIn];
  ps.sd_y = o[2 * kPolicyIn + 1];
  ps.ready = true;
  ps.dev_fresh = false;
  return GS_OK;
}

gs_status policy_save(gs_ctx_base* ctx, const char* path) {
  PolicyState& ps = ctx->policy;
  if (!ps.ready) P_FAIL(GS_EINVAL, "the learned policy has no parameters to save");
  FILE* f = std::fopen(path, "wb");
  if (!f) P_FAIL(GS_EINVAL, std::string("cannot open for writing: ") + path);
  std::vector<float> all((size_t)policy_param_floats());
  policy_get_params(ps, all.data());
  const uint32_t hdr[2] = {1u, (uint32_t)all.size()};
  const double cm[5] = {ps.c_pair, ps.c_dh, ps.c_dl, ps.c_h2l, ps.c_base};
  bool ok = std::fwrite(kParamMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
            std::fwrite(cm, sizeof(cm), 1, f) == 1 &&
            std::fwrite(all.data(), sizeof(float), all.size(), f) == all.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) P_FAIL(GS_EINVAL, std::string("write failed: ") + path);
  return GS_OK;
}

gs_status policy_load(gs_ctx_base* ctx, const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) P_FAIL(GS_EINVAL, std::string("cannot open: ") + path);
  char magic[8];
  uint32_t hdr[2];
  double cm[5];
  std::vector<float> all((size_t)policy_param_floats());
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kParamMagic, 8) == 0 &&
            std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 1u && hdr[1] == all.size() &&
            std::fread(cm, sizeof(cm), 1, f) == 1 &&
            std::fread(all.data(), sizeof(float), all.size(), f) == all.size();
  std::fclose(f);
  if (!ok) P_FAIL(GS_EINVAL, std::string("not a policy parameter file of this library: ") + path);
  for (double c : cm)
    if (!(c >= 0.0) || !std::isfinite(c)) P_FAIL(GS_EINVAL, "bad cost model in policy file");
  gs_status s = policy_set_params(ctx, all.data());
  if (s != GS_OK) return s;
  PolicyState& ps = ctx->policy;
  ps.c_pair = cm[0];
  ps.c_dh = cm[1];
  ps.c_dl = cm[2];
  ps.c_h2l = cm[3];
  ps.c_base = cm[4];
  return GS_OK;
}

gs_status policy_write_log(gs_ctx_base* ctx, const char* path) {
  PolicyState& ps = ctx->policy;
  FILE* f = std::fopen(path, "wb");
  if (!f) P_FAIL(GS_EINVAL, std::string("cannot open for writing: ") + path);
  const int64_t n = (int64_t)ps.log.size() / kPolicyRecord;
  const uint32_t hdr[2] = {1u, (uint32_t)kPolicyRecord};
  bool ok = std::fwrite(kLogMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
            std::fwrite(&n, sizeof(n), 1, f) == 1 &&
            std::fwrite(ps.log.data(), sizeof(float), ps.log.size(), f) == ps.log.size() &&
            std::fwrite(ps.log_keys.data(), sizeof(int32_t), ps.log_keys.size(), f) == ps.log_keys.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) P_FAIL(GS_EINVAL, std::string("write failed: ") + path);
  return GS_OK;
}

gs_status policy_read_log(gs_ctx_base* ctx, const char* path, std::vector<float>* rec) {
  FILE* f = std::fopen(path, "rb");
  if (!f) P_FAIL(GS_EINVAL, std::string("cannot open: ") + path);
  char magic[8];
  uint32_t hdr[2];
  int64_t n = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kLogMagic, 8) == 0 &&
            std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 1u && hdr[1] == (uint32_t)kPolicyRecord &&
            std::fread(&n, sizeof(n), 1, f) == 1 && n >= 0 && n <= INT32_MAX / 2;
  if (ok) {
    rec->resize((size_t)n * kPolicyRecord);
    ok = std::fread(rec->data(), sizeof(float), rec->size(), f) == rec->size();
  }
  std::fclose(f);
  if (!ok) P_FAIL(GS_EINVAL, std::string("not a policy log of this library: ") + path);
  return GS_OK;
}

}  // namespace gs
