// Orchestration of the dual-tree summation (sections 5-6): trees, moments,
// level-synchronous traversal, work lists, post-pass.
//
//   1. kd-trees of references (and of queries unless monochromatic)
//   2. raw Hermite moments to PLIMIT: leaves from points, H2H upward (Fig. 5)
//   3. traversal, one frontier level per iteration, all bandwidths at once:
//      decide (token rule) -> scan of per-segment counts -> emit (Figure 7)
//   4. the recorded work: DL then H2L into local coefficients, DH into
//      per-query sums, base cases into per-query sums
//   5. post-pass: Gest and L2L down the query tree, EVALL at the leaves
//      (Figure 8), results scattered to the caller's query order.
// The host reads back only the per-level totals it needs to size buffers.
#include <cstring>  // rocprim uses memset without including it
#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gs_host.h"
#include "gs_internal.h"
#include "gs_policy.h"
#include "gs_series.h"
#include "gs_traverse.h"
#include "gs_tree.h"

namespace gs {

// Event block of a dual-tree call (after the [n_h][6] decision counts): four
// counters, the token deposits and withdrawals (doubles), the order
// histogram [3][16] of the DH, DL and H2L pairs.
constexpr int kEvTok = 4;
constexpr int kEvHist = 6;
constexpr int kEvMfma = kEvHist + 3 * 16;
constexpr int kEvN = kEvMfma + 1;

namespace {

#define DT_FAIL(code, msg) \
  do {                     \
    ctx->err = (msg);      \
    return (code);         \
  } while (0)

#define DT_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t _e = (call);                                                           \
    if (_e != hipSuccess) {                                                           \
      (void)hipGetLastError();                                                        \
      ctx->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(_e); \
      return _e == hipErrorOutOfMemory ? GS_ENOMEM : GS_EDEVICE;                      \
    }                                                                                 \
  } while (0)

template <class T>
T* buf(gs_ctx_base* ctx, const std::string& name, size_t count, gs_status* st) {
  hipError_t e = hipSuccess;
  void* p = ctx->ws.get(name, count * sizeof(T), ctx, &e);
  if (!p) {
    ctx->err = "device allocation failed for workspace '" + name + "' (" +
               std::to_string(count * sizeof(T)) + " bytes)";
    *st = GS_ENOMEM;
  }
  return static_cast<T*>(p);
}

// Grow a named buffer to hold `need` elements, keeping its first `used`.
template <class T>
T* grow(gs_ctx_base* ctx, const std::string& name, size_t used, size_t need, hipStream_t s,
        gs_status* st) {
  if (ctx->inject_alloc_failure()) {
    ctx->err = "device allocation failed while growing '" + name + "'";
    *st = GS_ENOMEM;
    return nullptr;
  }
  Buf& b = ctx->ws.bufs[name];
  const size_t bytes = std::max<size_t>(need, 1) * sizeof(T);
  if (b.cap >= bytes) return static_cast<T*>(b.p);
  size_t cap = std::max(bytes, b.cap * 2);
  void* np = nullptr;
  if (hipMalloc(&np, cap) != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = "device allocation failed while growing '" + name + "'";
    *st = GS_ENOMEM;
    return nullptr;
  }
  if (b.p && used)
    (void)hipMemcpyAsync(np, b.p, used * sizeof(T), hipMemcpyDeviceToDevice, s);
  if (b.p) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(b.p);
  }
  b.p = np;
  b.cap = cap;
  return static_cast<T*>(np);
}

#define BUF(T, name, count)                                   \
  ({                                                          \
    gs_status _st = GS_OK;                                    \
    T* _p = buf<T>(ctx, std::string(name), (size_t)(count), &_st); \
    if (!_p) return _st;                                      \
    _p;                                                       \
  })

#define GROW(T, name, used, need)                                          \
  ({                                                                       \
    gs_status _st = GS_OK;                                                 \
    T* _p = grow<T>(ctx, std::string(name), (size_t)(used), (size_t)(need), st, &_st); \
    if (!_p) return _st;                                                   \
    _p;                                                                    \
  })

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ host tables

int plimit_table(int D) {
  switch (D) {
    case 1: return 10;
    case 2: return 8;
    case 3: return 6;
    case 4: return 5;
    case 5: return 4;
    case 6: return 2;
    default: return 1;
  }
}

uint64_t binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  if (k > n - k) k = n - k;
  uint64_t c = 1;
  for (int i = 1; i <= k; ++i) c = c * (uint64_t)(n - k + i) / (uint64_t)i;
  return c;
}

uint64_t ipow_sat(int b, int e) {
  uint64_t v = 1;
  for (int i = 0; i < e; ++i) {
    if (v > UINT64_MAX / (uint64_t)b) return UINT64_MAX;
    v *= (uint64_t)b;
  }
  return v;
}

uint64_t fact(int n) {
  uint64_t f = 1;
  for (int i = 2; i <= n; ++i) f *= (uint64_t)i;
  return f;
}

// C(D+p-1, D-1) / sqrt((floor(p/D)!)^{D-p'} (ceil(p/D)!)^{p'}), p' = p mod D (Lemma 4).
double bound_const(int D, int p) {
  const int q = p / D, pp = p % D;
  const int cq = pp ? q + 1 : q;
  uint64_t F = 1;
  for (int i = 0; i < D - pp; ++i) F *= fact(q);
  for (int i = 0; i < pp; ++i) F *= fact(cq);
  return (double)binom(D + p - 1, D - 1) / std::sqrt((double)F);
}

void degree_block(int D, int deg, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
  if (D == 1) {
    cur.push_back(deg);
    out.push_back(cur);
    cur.pop_back();
    return;
  }
  for (int first = deg; first >= 0; --first) {
    cur.push_back(first);
    degree_block(D - 1, deg - first, cur, out);
    cur.pop_back();
  }
}

}  // namespace

std::vector<std::vector<int>> multi_indices(int D, int p) {
  std::vector<std::vector<int>> out;
  std::vector<int> cur;
  for (int deg = 0; deg < p; ++deg) degree_block(D, deg, cur, out);
  return out;
}

namespace {

// All alpha in {0..m}^(D - cur.size()) completing cur, decreasing
// lexicographic order, kept when some component equals m.
void max_block(int D, int m, bool hit, std::vector<int>& cur, std::vector<std::vector<int>>& out) {
  if ((int)cur.size() == D) {
    if (hit) out.push_back(cur);
    return;
  }
  for (int v = m; v >= 0; --v) {
    cur.push_back(v);
    max_block(D, m, hit || v == m, cur, out);
    cur.pop_back();
  }
}

}  // namespace

// The O(p^D) set of section 2 (every alpha_d < p), ordered by the largest
// component so that order p is a prefix (its first p^D entries) of every
// larger order.
std::vector<std::vector<int>> tensor_indices(int D, int p) {
  std::vector<std::vector<int>> out;
  std::vector<int> cur;
  for (int m = 0; m < p; ++m) max_block(D, m, false, cur, out);
  return out;
}

// Largest order of the O(p^D) expansions: the O(D^p) limit, lowered until
// p^D terms fit the kernels' term bound.
int plimit_tensor(int D) {
  int p = plimit_table(D);
  while (p > 1 && ipow_sat(p, D) > (uint64_t)kMaxTerms) --p;
  return p;
}

namespace {

struct HostSeries {
  std::vector<int8_t> alpha;
  std::vector<int32_t> deg, nterms, h2h_start, l2l_start;
  std::vector<double> inv_fact, l2l_coef;
  std::vector<int2> h2h_pairs, l2l_pairs;
  int C = 0;
};

HostSeries make_series_tables(int D, int P, bool tensor) {
  HostSeries T;
  auto mis = tensor ? tensor_indices(D, P) : multi_indices(D, P);
  T.C = (int)mis.size();
  std::vector<uint64_t> afact(T.C);
  for (int i = 0; i < T.C; ++i) {
    int dg = 0;
    uint64_t f = 1;
    for (int d = 0; d < D; ++d) {
      T.alpha.push_back((int8_t)mis[i][d]);
      dg += mis[i][d];
      f *= fact(mis[i][d]);
    }
    T.deg.push_back(dg);
    afact[i] = f;
    T.inv_fact.push_back(1.0 / (double)f);
  }
  for (int p = 0; p <= P; ++p)
    T.nterms.push_back((int32_t)(tensor ? ipow_sat(p, D) : binom(D + p - 1, D)));
  auto index_of = [&](const std::vector<int>& a) {
    for (int i = 0; i < T.C; ++i)
      if (mis[i] == a) return i;
    return -1;
  };
  T.h2h_start.push_back(0);
  for (int g = 0; g < T.C; ++g) {
    for (int a = 0; a < T.C; ++a) {
      bool le = true;
      std::vector<int> diff(D);
      for (int d = 0; d < D; ++d) {
        if (mis[a][d] > mis[g][d]) le = false;
        diff[d] = mis[g][d] - mis[a][d];
      }
      if (le) T.h2h_pairs.push_back(make_int2(a, index_of(diff)));
    }
    T.h2h_start.push_back((int32_t)T.h2h_pairs.size());
  }
  T.l2l_start.push_back(0);
  for (int a = 0; a < T.C; ++a) {
    for (int b = 0; b < T.C; ++b) {
      bool ge = true;
      std::vector<int> diff(D);
      uint64_t df = 1;
      for (int d = 0; d < D; ++d) {
        if (mis[b][d] < mis[a][d]) ge = false;
        diff[d] = mis[b][d] - mis[a][d];
      }
      if (!ge) continue;
      for (int d = 0; d < D; ++d) df *= fact(diff[d]);
      T.l2l_pairs.push_back(make_int2(b, index_of(diff)));
      T.l2l_coef.push_back((double)afact[b] / ((double)afact[a] * (double)df));
    }
    T.l2l_start.push_back((int32_t)T.l2l_pairs.size());
  }
  return T;
}

// Order histogram of a work list: entries are (R << 4) | p.
__global__ void order_hist_kernel(const int32_t* __restrict__ ent, int64_t n, unsigned long long* __restrict__ hist) {
  __shared__ unsigned int part[16];
  if (threadIdx.x < 16) part[threadIdx.x] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&part[ent[i] & 15], 1u);
  __syncthreads();
  if (threadIdx.x < 16 && part[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)part[threadIdx.x]);
}

// Root pairs (h, root, root) of the bandwidths [h0, h0 + nh).
__global__ void init_level0_kernel(int h0, int nh, FrontierLevel f) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nh) return;
  f.h[k] = h0 + k;
  f.Q[k] = 0;
  f.off[k] = k;
  f.len[k] = 1;
  f.T[k] = 0.0;
  f.Lp[k] = 0.0;
  f.R[k] = 0;
  f.seg[k] = k;
}

__global__ void group_keys_kernel(int n, const int4* __restrict__ grp, int nQ,
                                  unsigned long long* __restrict__ key, int32_t* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = (unsigned long long)grp[i].x * (unsigned long long)nQ + (unsigned long long)grp[i].y;
  idx[i] = i;
}

// Host vector to device memory through a page-locked staging buffer of its
// own (name), so that the copy is asynchronous; the buffer is not reused
// before the call's final synchronisation.
template <class T>
hipError_t upload(gs_ctx_base* ctx, const char* name, const std::vector<T>& v, T* dst, hipStream_t s) {
  if (v.empty()) return hipSuccess;
  hipError_t e = hipSuccess;
  void* stage = ctx->ws.get_pinned(std::string("up_") + name, v.size() * sizeof(T), &e);
  if (!stage) return e;
  std::memcpy(stage, v.data(), v.size() * sizeof(T));
  return hipMemcpyAsync(dst, stage, v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

// Builds one tree into workspace buffers prefixed by `pre`.
static gs_status build_tree(gs_ctx_base* ctx, const char* pre, const double* xs, const double* w,
                            int64_t n, int D, int leaf_size, DevTree& t, hipStream_t st) {
  const std::string P(pre);
  const int64_t cap = tree_node_capacity(n, leaf_size);
  t.capacity = cap;
  t.begin = BUF(int32_t, P + "begin", cap);
  t.count = BUF(int32_t, P + "count", cap);
  t.left = BUF(int32_t, P + "left", cap);
  t.depth = BUF(int32_t, P + "depth", cap);
  t.parent = BUF(int32_t, P + "parent", cap);
  t.perm = BUF(int32_t, P + "perm", n);
  t.leaf_of_pos = BUF(int32_t, P + "leafpos", n);
  t.lo = BUF(double, P + "lo", cap * D);
  t.hi = BUF(double, P + "hi", cap * D);
  t.ctr = BUF(double, P + "ctr", cap * D);
  t.rinf = BUF(double, P + "rinf", cap);
  t.rad = BUF(double, P + "rad", cap);
  t.W = BUF(double, P + "W", cap);
  t.wmin = BUF(double, P + "wmin", cap);
  TreeBuildArgs a;
  a.n = n;
  a.D = D;
  a.leaf_size = leaf_size;
  a.xs = xs;
  a.w = w;
  a.ids = BUF(int32_t, "tb_ids", n);
  a.lists = BUF(int32_t, "tb_lists", n * (D + 1));
  a.lists_alt = BUF(int32_t, "tb_lists_alt", n * (D + 1));
  a.pos_node = BUF(int32_t, "tb_pos", n);
  a.pos_node_alt = BUF(int32_t, "tb_pos_alt", n);
  a.isleft = BUF(int32_t, "tb_isleft", n);
  a.flags = BUF(int32_t, "tb_flags", n * (D + 1));
  a.scan = BUF(int32_t, "tb_scan", n * (D + 1));
  a.splitdim = BUF(int32_t, "tb_splitdim", cap);
  a.sort_keys = BUF(double, "tb_sortkeys", n);
  a.temp_bytes = tree_sort_temp_bytes(n, D);
  a.temp = BUF(char, "tb_temp", a.temp_bytes);
  {
    hipError_t pe = hipSuccess;
    a.host_topo = static_cast<int32_t*>(ctx->ws.get_pinned(P + "topo", 5 * cap * sizeof(int32_t), &pe));
    if (!a.host_topo) DT_FAIL(GS_ENOMEM, "pinned host allocation failed for the tree topology");
  }
  hipError_t e = build_tree_device(a, t, t.level_begin, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ctx->err = std::string("tree build failed: ") + hipGetErrorString(e);
    return GS_EDEVICE;
  }
  return GS_OK;
}

static gs_status keep_tree(gs_ctx_base* ctx, const DevTree& t, int D, HostTree& h, hipStream_t st) {
  const int64_t nn = t.n_nodes, np = t.n_points;
  h.n_nodes = nn;
  h.n_points = np;
  h.perm.resize(np);
  h.begin.resize(nn);
  h.count.resize(nn);
  h.left.resize(nn);
  h.lo.resize(nn * D);
  h.hi.resize(nn * D);
  h.ctr.resize(nn * D);
  h.rinf.resize(nn);
  h.rad.resize(nn);
  h.W.resize(nn);
  h.wmin.resize(nn);
  auto cp = [&](auto& v, const auto* src) {
    return hipMemcpyAsync(v.data(), src, v.size() * sizeof(v[0]), hipMemcpyDeviceToHost, st);
  };
  DT_HIP(cp(h.perm, t.perm));
  DT_HIP(cp(h.begin, t.begin));
  DT_HIP(cp(h.count, t.count));
  DT_HIP(cp(h.left, t.left));
  DT_HIP(cp(h.lo, t.lo));
  DT_HIP(cp(h.hi, t.hi));
  DT_HIP(cp(h.ctr, t.ctr));
  DT_HIP(cp(h.rinf, t.rinf));
  DT_HIP(cp(h.rad, t.rad));
  DT_HIP(cp(h.W, t.W));
  DT_HIP(cp(h.wmin, t.wmin));
  DT_HIP(hipStreamSynchronize(st));
  h.valid = true;
  return GS_OK;
}

void finish_dualtree_stats(gs_ctx_base* ctx) {
  const unsigned long long* hc = ctx->stats_pending;
  if (!hc) return;
  const int n_h = ctx->stats_pending_nh;
  gs_stats& S = ctx->stats;
  for (int k = 0; k < n_h * 6; ++k) {
    ctx->pair_counts[k] = (int64_t)hc[k];
    S.pairs[k % 6] += (int64_t)hc[k];
  }
  S.base_pair_evals = (int64_t)hc[n_h * 6];
  S.base_dist_evals = (int64_t)hc[n_h * 6 + 1];
  S.policy_calls = (int64_t)hc[n_h * 6 + 2];
  S.policy_overrides = (int64_t)hc[n_h * 6 + 3];
  std::memcpy(&S.tokens_deposited, hc + n_h * 6 + kEvTok, sizeof(double));
  std::memcpy(&S.tokens_withdrawn, hc + n_h * 6 + kEvTok + 1, sizeof(double));
  for (int x = 0; x < 3; ++x)
    for (int p = 0; p < 16; ++p) S.p_hist[x][p] = (int64_t)hc[n_h * 6 + kEvHist + 16 * x + p];
  S.base_mfma_pair_evals = (int64_t)hc[n_h * 6 + kEvMfma];
  ctx->stats_pending = nullptr;
}

gs_status run_dualtree(gs_ctx_base* ctx, const DeviceInputs& in, const std::vector<double>& hs,
                       double eps, const gs_options& opt, double* G_dev) {
  hipStream_t st = ctx->stream;
  const int D = in.D;
  const int64_t N = in.N, Mq = in.M;
  const int n_h = (int)hs.size();
  const bool tensor = opt.method == GS_DFTO;
  const bool use_fmm = opt.method == GS_DUALTREE || tensor;
  const bool use_tokens = opt.method != GS_DFD;
  int P = opt.plimit > 0 ? opt.plimit : (tensor ? plimit_tensor(D) : plimit_table(D));
  if (P > kMaxPlimit) DT_FAIL(GS_EINVAL, "plimit must be <= 10");
  if (!use_fmm) P = 1;
  if (tensor && ipow_sat(P, D) > (uint64_t)kMaxTerms)
    DT_FAIL(GS_EINVAL, "plimit too large for this dimension (GS_DFTO needs p^D <= 286)");
  if ((int64_t)binom(D + P - 1, D) > kMaxTerms || D * P > 64)
    DT_FAIL(GS_EINVAL, "plimit too large for this dimension (need C(D+p-1,D) <= 286 and D*p <= 64)");
  gs_stats& S = ctx->stats;
  S.plimit = P;
  double t0 = now_ms();

  // 1. Trees.
  KernelTimer ktree(ctx, ctx->kernel_timing, GS_K_TREE, st);
  DevTree rt, qt_own;
  gs_status s = build_tree(ctx, "rt_", in.r_soa, in.w, N, D, opt.leaf_size, rt, st);
  if (s != GS_OK) return s;
  DevTree* qtp = &rt;
  if (!in.mono) {
    s = build_tree(ctx, "qt_", in.q_soa, nullptr, Mq, D, opt.leaf_size, qt_own, st);
    if (s != GS_OK) return s;
    qtp = &qt_own;
  }
  DevTree& qt = *qtp;
  const int nR = (int)rt.n_nodes, nQ = (int)qt.n_nodes;
  double* xr_perm = BUF(double, "xr_perm", N * D);
  double* wr_perm = BUF(double, "wr_perm", N);
  DT_HIP(launch_gather_rows(in.r_aos, rt.perm, N, D, xr_perm, st));
  DT_HIP(launch_gather(in.w, rt.perm, N, wr_perm, st));
  double* xq_perm = xr_perm;
  if (!in.mono) {
    xq_perm = BUF(double, "xq_perm", Mq * D);
    DT_HIP(launch_gather_rows(in.q_aos, qt.perm, Mq, D, xq_perm, st));
  }
  if (opt.node_bounds == 1) {
    DT_HIP(launch_node_radius(rt, rt.n_nodes, xr_perm, D, st));
    if (!in.mono) DT_HIP(launch_node_radius(qt, qt.n_nodes, xq_perm, D, st));
  }
  unsigned long long* wmax_bits = BUF(unsigned long long, "wmax_bits", 1);
  DT_HIP(launch_max_positive(in.w, N, wmax_bits, st));
  ktree.stop(st, 1);
  double t1 = now_ms();
  S.t_tree_ms = t1 - t0;

  // 2. Series tables and moments.
  HostSeries hsr = make_series_tables(D, P, tensor);
  const int C = hsr.C;
  SeriesTables T;
  T.D = D;
  T.P = P;
  T.C = C;
  {
    int8_t* alpha = BUF(int8_t, "ts_alpha", hsr.alpha.size());
    int32_t* deg = BUF(int32_t, "ts_deg", hsr.deg.size());
    double* invf = BUF(double, "ts_invf", hsr.inv_fact.size());
    int32_t* nterms = BUF(int32_t, "ts_nterms", hsr.nterms.size());
    int32_t* hs0 = BUF(int32_t, "ts_h2hs", hsr.h2h_start.size());
    int2* hp = BUF(int2, "ts_h2hp", hsr.h2h_pairs.size());
    int32_t* ls0 = BUF(int32_t, "ts_l2ls", hsr.l2l_start.size());
    int2* lp = BUF(int2, "ts_l2lp", hsr.l2l_pairs.size());
    double* lc = BUF(double, "ts_l2lc", hsr.l2l_coef.size());
    DT_HIP(upload(ctx, "alpha", hsr.alpha, alpha, st));
    DT_HIP(upload(ctx, "deg", hsr.deg, deg, st));
    DT_HIP(upload(ctx, "invf", hsr.inv_fact, invf, st));
    DT_HIP(upload(ctx, "nterms", hsr.nterms, nterms, st));
    DT_HIP(upload(ctx, "hs0", hsr.h2h_start, hs0, st));
    DT_HIP(upload(ctx, "hp", hsr.h2h_pairs, hp, st));
    DT_HIP(upload(ctx, "ls0", hsr.l2l_start, ls0, st));
    DT_HIP(upload(ctx, "lp", hsr.l2l_pairs, lp, st));
    DT_HIP(upload(ctx, "lc", hsr.l2l_coef, lc, st));
    T.alpha = alpha;
    T.deg = deg;
    T.inv_fact = invf;
    T.nterms = nterms;
    T.h2h_start = hs0;
    T.h2h_pairs = hp;
    T.l2l_start = ls0;
    T.l2l_pairs = lp;
    T.l2l_coef = lc;
  }
  NodeView rv{rt.begin, rt.count, rt.left, rt.ctr, rt.lo, rt.hi};
  NodeView qv{qt.begin, qt.count, qt.left, qt.ctr, qt.lo, qt.hi};
  double* Mom = nullptr;
  if (use_fmm) {
    Mom = BUF(double, "moments", (int64_t)nR * C);
    // Only the expansions read the moments, and they run on the side stream
    // (below), so the moments go there too, beside the traversal; each
    // bandwidth chunk joins the side stream back before it returns.
    hipStream_t sm = st;
    if (!opt.log_pairs && ctx->side) {
      DT_HIP(hipEventRecord(ctx->fork_ev, st));
      DT_HIP(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
      sm = ctx->side;
    }
    KernelTimer km(ctx, ctx->kernel_timing, GS_K_MOMENTS, sm);
    if (series_fast_available(D, P, tensor))
      DT_HIP(launch_p2m_fast(D, P, tensor, rv, nR, xr_perm, wr_perm, Mom, sm));
    else
      DT_HIP(launch_p2m(T, rv, nR, xr_perm, wr_perm, Mom, sm));
    for (int lv = (int)rt.level_begin.size() - 2; lv >= 0; --lv)
      DT_HIP(series_fast_available(D, P, tensor)
                 ? launch_h2h_level_fast(D, P, tensor, rv, rt.level_begin[lv], rt.level_begin[lv + 1], Mom, sm)
                 : launch_h2h_level(T, rv, rt.level_begin[lv], rt.level_begin[lv + 1], Mom, sm));
    km.stop(sm, (int)rt.level_begin.size());
  }
  double t2 = now_ms();
  S.t_moments_ms = t2 - t1;

  // Per-bandwidth constants.  The three reciprocals enter pruning decisions
  // and are formed exactly like this by any reproduction of the decisions.
  std::vector<double> h_inv2h2(n_h), h_inv4h2(n_h), h_invh(n_h), h_sc(n_h);
  std::vector<float> h_s2(n_h);
  for (int k = 0; k < n_h; ++k) {
    const double h = hs[k];
    h_inv2h2[k] = 1.0 / (2.0 * h * h);
    h_inv4h2[k] = 0.5 * h_inv2h2[k];
    h_invh[k] = 1.0 / h;
    h_sc[k] = 1.0 / std::sqrt(2.0 * h * h);
    h_s2[k] = (float)(1.4426950408889634 / (2.0 * h * h));
  }
  double* d_inv2h2 = BUF(double, "h_inv2h2", n_h);
  double* d_inv4h2 = BUF(double, "h_inv4h2", n_h);
  double* d_invh = BUF(double, "h_invh", n_h);
  double* d_sc = BUF(double, "h_sc", n_h);
  float* d_s2 = BUF(float, "h_s2", n_h);
  double* d_hs = BUF(double, "h_hs", n_h);
  DT_HIP(upload(ctx, "d_hs", hs, d_hs, st));
  DT_HIP(upload(ctx, "d_inv2h2", h_inv2h2, d_inv2h2, st));
  DT_HIP(upload(ctx, "d_inv4h2", h_inv4h2, d_inv4h2, st));
  DT_HIP(upload(ctx, "d_invh", h_invh, d_invh, st));
  DT_HIP(upload(ctx, "d_sc", h_sc, d_sc, st));
  DT_HIP(upload(ctx, "d_s2", h_s2, d_s2, st));

  DecideConst dc;
  std::memset(&dc, 0, sizeof(dc));
  dc.D = D;
  dc.P = P;
  dc.mono = in.mono ? 1 : 0;
  dc.use_tokens = use_tokens ? 1 : 0;
  dc.use_fmm = use_fmm ? 1 : 0;
  dc.eps_alg = (1.0 - opt.eps_round_share) * eps;
  dc.tensor = tensor ? 1 : 0;
  dc.fmm_mask = (opt.fmm_mask & 7) ? (opt.fmm_mask & 7) : 7;
  const bool use_policy = use_fmm && opt.policy == GS_LEARNED;
  const bool log_pairs = use_fmm && opt.log_pairs;
  dc.policy = use_policy ? 1 : 0;
  dc.log_feas = log_pairs ? 1 : 0;
  dc.node_bounds = opt.node_bounds;
  dc.explore = opt.log_explore;
  PolicyDevModel pmodel;
  if (use_policy) {
    s = policy_device_model(ctx, &pmodel);
    if (s != GS_OK) return s;
  }
  for (int p = 1; p <= P; ++p) {
    dc.bconst[p] = bound_const(D, p);
    dc.binomD[p] = (double)binom(D + p - 1, D);
  }
  // Cramer's classical constant 1.086435..., rounded up
  dc.kc = 1.09;
  for (int n = 0; n <= kMaxPlimit; ++n) {
    dc.isf[n] = 1.0 / std::sqrt((double)fact(n));
    dc.isq[n] = 1.0 / std::sqrt((double)(n + 1));
  }
  {
    auto sat = [](uint64_t v) { return v > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)v; };
    auto mul = [](int64_t a, int64_t b) {
      int64_t r;
      return __builtin_mul_overflow(a, b, &r) ? INT64_MAX : r;
    };
    for (int p = 0; p <= kMaxPlimit; ++p) {
      dc.cterm[p] = tensor ? mul(D, sat(ipow_sat(p, D))) : sat(ipow_sat(D, p + 1));
      dc.ch2l[p] = tensor ? mul(D, sat(ipow_sat(p, 2 * D))) : sat(ipow_sat(D, 2 * p + 1));
    }
  }

  // Per (h, query node) and per (h, query point) state.
  double* Gest = BUF(double, "Gest", (int64_t)n_h * nQ);
  int32_t* pL = BUF(int32_t, "pL", (int64_t)n_h * nQ);
  double* lco = use_fmm ? BUF(double, "lco", (int64_t)n_h * nQ * C) : nullptr;
  double* gx = BUF(double, "gx", (int64_t)n_h * Mq);
  double* gdh = BUF(double, "gdh", (int64_t)n_h * Mq);
  // [n_h][6] decisions per type, then the call's event block (kEvN slots):
  // four counters (base point-pair evaluations, base distance evaluations,
  // policy consultations, policy overrides), the token deposits and
  // withdrawals (two doubles), the order histogram [3][16] of the DH, DL and
  // H2L pairs; then the block's copy taken at the start of each chunk.
  unsigned long long* hcount = BUF(unsigned long long, "hcount", (int64_t)n_h * 6 + 2 * kEvN);
  unsigned long long* chunk_ev = hcount + n_h * 6;
  dc.tok = use_tokens ? reinterpret_cast<double*>(chunk_ev + kEvTok) : nullptr;
  DT_HIP(hipMemsetAsync(Gest, 0, sizeof(double) * n_h * nQ, st));
  DT_HIP(hipMemsetAsync(pL, 0, sizeof(int32_t) * n_h * nQ, st));
  if (lco) DT_HIP(hipMemsetAsync(lco, 0, sizeof(double) * n_h * nQ * C, st));
  DT_HIP(hipMemsetAsync(gx, 0, sizeof(double) * n_h * Mq, st));
  DT_HIP(hipMemsetAsync(gdh, 0, sizeof(double) * n_h * Mq, st));
  DT_HIP(hipMemsetAsync(hcount, 0, sizeof(unsigned long long) * (n_h * 6 + 2 * kEvN), st));
  float* rec = nullptr;  // base-case reference records, built on first use
  bool rec_ready = false;
  BaseRecordsArgs ra;

  TreeView qtv{qt.lo, qt.hi, qt.rinf, qt.W, qt.wmin, qt.count, qt.left, qt.ctr, qt.rad};
  TreeView rtv{rt.lo, rt.hi, rt.rinf, rt.W, rt.wmin, rt.count, rt.left, rt.ctr, rt.rad};
  auto level_bufs = [&](int which, int64_t nseg, int64_t npair, FrontierLevel& f) -> gs_status {
    const std::string p = which ? "f1_" : "f0_";
    f.h = BUF(int32_t, p + "h", nseg);
    f.Q = BUF(int32_t, p + "Q", nseg);
    f.off = BUF(int32_t, p + "off", nseg);
    f.len = BUF(int32_t, p + "len", nseg);
    f.T = BUF(double, p + "T", nseg);
    f.Lp = BUF(double, p + "Lp", nseg);
    f.R = BUF(int32_t, p + "R", npair);
    f.seg = BUF(int32_t, p + "seg", npair);
    f.first = BUF(int32_t, p + "first", nseg);
    return GS_OK;
  };
  const char* tname[4] = {"dh", "dl", "h2l", "base"};
  const int64_t max_frontier =
      opt.max_frontier > 0 ? std::min<int64_t>(opt.max_frontier, kMaxFrontier) : kMaxFrontier;
  double t_trav = 0.0, t_work = 0.0;
  int64_t peak = 0;
  int max_level = 0;
  PolicyTreeView pqt{qt.lo, qt.hi, qt.rinf, qt.count, qt.left};
  PolicyTreeView prt{rt.lo, rt.hi, rt.rinf, rt.count, rt.left};

  // Steps 3 and 4 for the bandwidths [hc0, hc1).  Bandwidths never interact
  // in the traversal, so any split of the sweep makes the same decisions.
  // Sets *retry (and changes nothing the final result depends on) when the
  // frontier or a work list outgrows 32-bit indexing or device memory before
  // any work kernel ran; the caller then halves the chunk.
  auto run_chunk = [&](int hc0, int hc1, bool* retry) -> gs_status {
    const int nh = hc1 - hc0;
    *retry = false;
    const size_t trace0 = ctx->trace.size();
    auto overflow = [&]() -> gs_status {
      if (nh == 1)
        DT_FAIL(GS_EOVERFLOW, "the frontier of a single bandwidth exceeds max_frontier (or 2^30) "
                              "pairs, or a work list exceeds 2^30 entries");
      *retry = true;
      // Undo the chunk's decisions: lower-bound sums, counters and trace.
      DT_HIP(hipMemsetAsync(Gest + (int64_t)hc0 * nQ, 0, sizeof(double) * nh * nQ, st));
      DT_HIP(hipMemsetAsync(hcount + hc0 * 6, 0, sizeof(unsigned long long) * nh * 6, st));
      DT_HIP(hipMemcpyAsync(chunk_ev, chunk_ev + kEvN, kEvN * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                            st));
      DT_HIP(hipStreamSynchronize(st));
      ctx->trace.resize(trace0);
      ctx->trace_feat.resize(trace0 / 6 * kPolicyIn);
      ctx->trace_feas.resize(trace0 / 6);
      return GS_OK;
    };
    // A failed allocation during the traversal is retried with fewer bandwidths.
#define CHUNK_ALLOC(expr)                                  \
  do {                                                     \
    gs_status _s = (expr);                                 \
    if (_s == GS_ENOMEM && nh > 1) return overflow();      \
    if (_s != GS_OK) return _s;                            \
  } while (0)
    const double ta = now_ms();
    // the event counters run over the whole call; a retried chunk restores them
    DT_HIP(hipMemcpyAsync(chunk_ev + kEvN, chunk_ev, kEvN * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                          st));
    FrontierLevel cur, nxt;
    int64_t nseg = nh, npair = nh;
    CHUNK_ALLOC(level_bufs(0, nseg, npair, cur));
    hipLaunchKernelGGL(init_level0_kernel, dim3((unsigned)ceil_div(nh, 64)), dim3(64), 0, st, hc0, nh, cur);
    DT_HIP(hipGetLastError());
    WorkLists wl;
    int64_t used_ent[4] = {0, 0, 0, 0}, used_grp[4] = {0, 0, 0, 0}, used_slc[2] = {0, 0};
    auto grow_lists = [&](const int64_t* add_ent, const int64_t* add_grp, const int64_t* add_slc) -> gs_status {
      for (int x = 0; x < 4; ++x) {
        wl.ent[x] = GROW(int32_t, std::string("wl_ent_") + tname[x], used_ent[x], used_ent[x] + add_ent[x]);
        wl.grp[x] = GROW(int4, std::string("wl_grp_") + tname[x], used_grp[x], used_grp[x] + add_grp[x]);
      }
      wl.dh_first = GROW(int32_t, "wl_dh_first", used_grp[0], used_grp[0] + add_grp[0]);
      wl.dl_first = GROW(int2, "wl_dl_first", used_grp[1], used_grp[1] + add_grp[1]);
      wl.dl_cpre = GROW(int32_t, "wl_dl_cpre", used_ent[1], used_ent[1] + add_ent[1]);
      wl.dh_slice = GROW(int4, "wl_dh_slice", used_slc[0], used_slc[0] + add_slc[0]);
      wl.dl_slice = GROW(int4, "wl_dl_slice", used_slc[1], used_slc[1] + add_slc[1]);
      return GS_OK;
    };
    {
      const int64_t e0[4] = {1024, 1024, 1024, 1024}, g0[4] = {256, 256, 256, 256}, s0[2] = {256, 256};
      CHUNK_ALLOC(grow_lists(e0, g0, s0));
    }
    int level = 0, which = 0;
    SegCount* seg_tot = nullptr;  // page-locked: the per-level readback
    {
      hipError_t pe = hipSuccess;
      seg_tot = static_cast<SegCount*>(ctx->ws.get_pinned("seg_tot", sizeof(SegCount), &pe));
      if (!seg_tot) DT_FAIL(GS_ENOMEM, "pinned host allocation failed for the frontier counts");
    }
    int64_t nfirst = 0;  // long segments of the current level
    std::vector<int64_t> dh_level_begin;  // first DH group of each traversal level
    std::vector<int64_t> dh_slice_begin;  // first DH slice of each traversal level
    std::vector<int32_t> tr_h, tr_Q, tr_off, tr_len, tr_R;
    std::vector<int8_t> tr_code, tr_p;
    std::vector<float> tr_feat;
    std::vector<int16_t> tr_feas;
    while (nseg > 0) {
      peak = std::max(peak, npair);
      int8_t* code;
      int8_t* pord;
      SegCount *cnt, *incl;
      double* prep;
      void* temp;
      float4* scores = nullptr;
      float* pfeat = nullptr;
      int16_t* pfeas = nullptr;
      const size_t tb = scan_counts_temp_bytes((int)nseg);
      double* ff_d2 = nullptr;
      int32_t* ff_R = nullptr;
      const bool far_first = opt.pair_order == GS_ORDER_FAR_FIRST && level > 0;
      CHUNK_ALLOC(([&]() -> gs_status {
        if (far_first) {
          ff_d2 = BUF(double, "ff_d2", npair);
          ff_R = BUF(int32_t, "ff_R", npair);
        }
        code = BUF(int8_t, "p_code", npair);
        pord = BUF(int8_t, "p_ord", npair);
        cnt = BUF(SegCount, "seg_cnt", nseg);
        incl = BUF(SegCount, "seg_incl", nseg);
        prep = BUF(double, "p_prep", 5 * npair);
        temp = BUF(char, "scan_temp", tb);
        if (use_policy) scores = BUF(float4, "p_scores", npair);
        if (log_pairs) {
          pfeat = BUF(float, "p_feat", npair * kPolicyIn);
          pfeas = BUF(int16_t, "p_feas", npair);
        }
        return GS_OK;
      })());
      const PolicyPairs pp{cur.h, cur.Q, cur.seg, cur.R, d_hs, d_invh};
      {
        KernelTimer kt(ctx, ctx->kernel_timing, GS_K_DECIDE, st);
        // best-first walk of each query node's list (option pair_order)
        if (far_first) DT_HIP(launch_far_first_order((int)npair, cur, qtv, rtv, D, dc.node_bounds, ff_d2, ff_R, st));
        if (use_policy) DT_HIP(launch_policy_infer_pairs((int)npair, pp, pqt, prt, D, pmodel, scores, st));
        if (log_pairs) DT_HIP(launch_policy_features((int)npair, pp, pqt, prt, D, pfeat, st));
        DT_HIP(launch_decide((int)nseg, (int)nfirst, cur, qtv, rtv, d_inv2h2, d_inv4h2, d_invh, nQ, dc, code, pord,
                             Gest, cnt, scores, pfeas, prep, (int)npair, st));
        DT_HIP(scan_counts((int)nseg, cnt, incl, temp, tb, st));
        kt.stop(st, 2 + (use_policy ? 1 : 0) + (log_pairs ? 1 : 0));
      }
      DT_HIP(hipMemcpyAsync(seg_tot, incl + (nseg - 1), sizeof(SegCount), hipMemcpyDeviceToHost, st));
      DT_HIP(hipStreamSynchronize(st));
      const SegCount tot = *seg_tot;
      if (opt.keep_trace) {
        tr_h.resize(nseg);
        tr_Q.resize(nseg);
        tr_off.resize(nseg);
        tr_len.resize(nseg);
        tr_R.resize(npair);
        tr_code.resize(npair);
        tr_p.resize(npair);
        DT_HIP(hipMemcpyAsync(tr_h.data(), cur.h, nseg * 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipMemcpyAsync(tr_Q.data(), cur.Q, nseg * 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipMemcpyAsync(tr_off.data(), cur.off, nseg * 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipMemcpyAsync(tr_len.data(), cur.len, nseg * 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipMemcpyAsync(tr_R.data(), cur.R, npair * 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipMemcpyAsync(tr_code.data(), code, npair, hipMemcpyDeviceToHost, st));
        DT_HIP(hipMemcpyAsync(tr_p.data(), pord, npair, hipMemcpyDeviceToHost, st));
        if (log_pairs) {
          tr_feat.resize(npair * kPolicyIn);
          tr_feas.resize(npair);
          DT_HIP(hipMemcpyAsync(tr_feat.data(), pfeat, npair * kPolicyIn * sizeof(float),
                                hipMemcpyDeviceToHost, st));
          DT_HIP(hipMemcpyAsync(tr_feas.data(), pfeas, npair * sizeof(int16_t), hipMemcpyDeviceToHost, st));
        }
        DT_HIP(hipStreamSynchronize(st));
        for (int64_t k = 0; k < nseg; ++k)
          for (int j = 0; j < tr_len[k]; ++j) {
            const int64_t o = tr_off[k] + j;
            const int32_t r6[6] = {tr_h[k], level, tr_Q[k], tr_R[o], tr_code[o], tr_p[o]};
            ctx->trace.insert(ctx->trace.end(), r6, r6 + 6);
            if (log_pairs) {
              ctx->trace_feat.insert(ctx->trace_feat.end(), tr_feat.begin() + o * kPolicyIn,
                                     tr_feat.begin() + (o + 1) * kPolicyIn);
              ctx->trace_feas.push_back(tr_feas[o]);
            }
          }
      }
      const int64_t nseg2 = tot.v[1], npair2 = tot.v[0];
      bool too_big = npair2 > max_frontier || nseg2 > max_frontier;
      for (int x = 0; x < 4; ++x)
        too_big = too_big || used_ent[x] + tot.v[2 + x] > kMaxFrontier ||
                  used_grp[x] + tot.v[6 + x] > kMaxFrontier;
      for (int x = 0; x < 2; ++x) too_big = too_big || used_slc[x] + tot.v[15 + x] > kMaxFrontier;
      if (too_big) return overflow();
      dh_level_begin.push_back(used_grp[0]);
      dh_slice_begin.push_back(used_slc[0]);
      CHUNK_ALLOC(grow_lists(tot.v + 2, tot.v + 6, tot.v + 15));
      LevelOffsets lo;
      for (int x = 0; x < 4; ++x) {
        lo.ent[x] = (int32_t)used_ent[x];
        lo.grp[x] = (int32_t)used_grp[x];
      }
      for (int x = 0; x < 2; ++x) lo.slc[x] = (int32_t)used_slc[x];
      CHUNK_ALLOC(level_bufs(1 - which, nseg2, npair2, nxt));
      {
        KernelTimer kt(ctx, ctx->kernel_timing, GS_K_DECIDE, st);
        DT_HIP(launch_emit((int)nseg, cur, nxt, qt.left, rt.left, code, pord, cnt, incl, rt.count, wl,
                           lo, hcount, chunk_ev, st));
        kt.stop(st, 1);
      }
      for (int x = 0; x < 4; ++x) {
        used_ent[x] += tot.v[2 + x];
        used_grp[x] += tot.v[6 + x];
      }
      for (int x = 0; x < 2; ++x) used_slc[x] += tot.v[15 + x];
      std::swap(cur, nxt);
      which = 1 - which;
      nseg = nseg2;
      npair = npair2;
      nfirst = tot.v[17];
      ++level;
    }
    // orders of the chunk's DH, DL and H2L pairs (the work-list entries)
    for (int x = 0; x < 3 && use_fmm; ++x)
      if (used_ent[x] > 0) {
        hipLaunchKernelGGL(order_hist_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(used_ent[x], 256), 1024)),
                           dim3(256), 0, st, wl.ent[x], used_ent[x], chunk_ev + kEvHist + 16 * x);
        DT_HIP(hipGetLastError());
      }
    const double tb0 = now_ms();
    t_trav += tb0 - ta;
    max_level = std::max(max_level, level);
    dh_level_begin.push_back(used_grp[0]);
    dh_slice_begin.push_back(used_slc[0]);

    // 4. Work.  Every scratch buffer is taken before the first work kernel,
    // so a failed allocation can still be retried.
    SortedGroups sg[3];
    unsigned long long* gkey[3] = {};
    int32_t* gidx[3] = {};
    size_t gsort_bytes = 0;
    BaseFusedArgs ba;
    const bool any_base = used_grp[3] > 0;
    const bool fast = use_fmm && series_fast_available(D, P, tensor);
    double* dh_part = nullptr;
    double* dl_part = nullptr;
    int32_t* dl_part_p = nullptr;
    double* h2l_part = nullptr;
    int32_t* h2l_part_p = nullptr;
    CHUNK_ALLOC(([&]() -> gs_status {
      if (fast) {
        // partial sums of the sliced DH and DL kernels
        int64_t dh_need = 0;
        for (size_t lv = 0; lv + 1 < dh_slice_begin.size(); ++lv) {
          const int depth_max = lv < qt.level_max.size() ? qt.level_max[lv] : 0;
          const int64_t cy = ceil_div(std::max(depth_max, opt.leaf_size), 64);
          dh_need = std::max(dh_need, (dh_slice_begin[lv + 1] - dh_slice_begin[lv]) * cy * 64);
        }
        if (dh_need) dh_part = BUF(double, "dh_part", dh_need);
        if (used_slc[1]) {
          dl_part = BUF(double, "dl_part", used_slc[1] * series_terms(D, P, tensor));
          dl_part_p = BUF(int32_t, "dl_part_p", used_slc[1]);
        }
        if (used_grp[2]) {
          h2l_part = BUF(double, "h2l_part", used_grp[2] * series_terms(D, P, tensor));
          h2l_part_p = BUF(int32_t, "h2l_part_p", used_grp[2]);
        }
      }
      for (int x = 1; x < 3; ++x) {
        const int n = (int)used_grp[x];
        sg[x].n = n;
        sg[x].grp = wl.grp[x];
        if (n == 0 || !use_fmm) continue;
        gkey[x] = BUF(unsigned long long, std::string("g_key_") + tname[x], n);
        sg[x].key = BUF(unsigned long long, std::string("g_skey_") + tname[x], n);
        gidx[x] = BUF(int32_t, std::string("g_idx_") + tname[x], n);
        sg[x].order = BUF(int32_t, std::string("g_sidx_") + tname[x], n);
        size_t bytes = 0;
        DT_HIP(rocprim::radix_sort_pairs((void*)nullptr, bytes, gkey[x], (unsigned long long*)nullptr,
                                         gidx[x], (int32_t*)nullptr, (unsigned)n, 0, 64, st));
        gsort_bytes = std::max(gsort_bytes, bytes);
      }
      if (!any_base) return GS_OK;
      const int64_t ne = used_ent[3];
      if (!rec) {
        ra.xr_perm = xr_perm;
        ra.wr_perm = wr_perm;
        ra.leaf_of_pos = rt.leaf_of_pos;
        ra.begin = rt.begin;
        ra.count = rt.count;
        ra.left = rt.left;
        ra.rctr = rt.ctr;
        ra.n = N;
        ra.D = D;
        ra.n_nodes = nR;
        ra.wmax_bits = wmax_bits;
        ra.padded = BUF(int32_t, "rec_pad", nR);
        ra.rec_off = BUF(int32_t, "rec_off", nR);
        ra.rec_capacity = base_records_capacity(N, nR);
        ra.temp_bytes = base_records_temp_bytes(nR);
        ra.temp = BUF(char, "rec_temp", ra.temp_bytes);
        rec = BUF(float, "base_rec", ra.rec_capacity * base_record_stride(D));
        ra.rec = rec;
      }
      if (base_uses_mfma(D) && !ra.mrec) {
        // set together once all three are allocated: a failed request here is
        // retried whole
        const int64_t groups = base_mfma_groups_capacity(N, nR);
        float* mrec = BUF(float, "base_mrec", groups * base_mfma_group_floats(D));
        int32_t* mgrp_off = BUF(int32_t, "base_mgrp_off", nR);
        float* rmax2 = BUF(float, "base_rmax2", nR);
        ra.mgroups_capacity = groups;
        ra.mgrp_off = mgrp_off;
        ra.rmax2 = rmax2;
        ra.mrec = mrec;
      }
      ba.grp = wl.grp[3];
      ba.n_groups = (int)used_grp[3];
      ba.ent = wl.ent[3];
      ba.n_entries = ne;
      ba.n_qnodes = nQ;
      ba.n_rnodes = nR;
      ba.n_hblocks = (n_h + kBaseHB - 1) / kBaseHB;
      ba.hc0 = hc0;
      ba.hc1 = hc1;
      ba.qt = qv;
      ba.rt = rv;
      ba.xq_perm = xq_perm;
      ba.rec = rec;
      ba.rec_off = ra.rec_off;
      ba.mrec = ra.mrec;
      ba.mgrp_off = ra.mgrp_off;
      ba.rmax2 = ra.rmax2;
      ba.mfma_evals = chunk_ev + kEvMfma;
      ba.max_leaf = opt.leaf_size;
      ba.D = D;
      ba.Mq = (int)Mq;
      ba.s2 = d_s2;
      ba.wmax_bits = wmax_bits;
      ba.gx = gx;
      ba.dist_evals = chunk_ev + 1;
      ba.key = BUF(unsigned long long, "bf_key", ne);
      ba.key_sorted = BUF(unsigned long long, "bf_skey", ne);
      ba.ukey = BUF(unsigned long long, "bf_ukey", ne);
      ba.bit = BUF(BaseMask, "bf_bit", ne);
      ba.bit_sorted = BUF(BaseMask, "bf_sbit", ne);
      ba.umask = BUF(BaseMask, "bf_umask", ne);
      ba.flag = BUF(int32_t, "bf_flag", ne);
      ba.pos = BUF(int32_t, "bf_pos", ne);
      ba.mflag = BUF(int32_t, "bf_mflag", ne);
      ba.mpos = BUF(int32_t, "bf_mpos", ne);
      ba.run_start = BUF(int32_t, "bf_runs", ne + 1);
      ba.slices = BUF(int4, "bf_slices", base_max_slices(ne));
      const int nslots = base_partial_slots(opt.leaf_size);
      ba.slots = BUF(int4, "bf_slots", nslots);
      ba.partial = BUF(double, "bf_partial", base_partial_doubles(opt.leaf_size));
      ba.counters = BUF(int32_t, "bf_counters", 8);
      {
        hipError_t pe = hipSuccess;
        ba.host_counters = static_cast<int32_t*>(ctx->ws.get_pinned("bf_counters", 4 * sizeof(int32_t), &pe));
        if (!ba.host_counters) return GS_ENOMEM;
      }
      ba.temp_bytes = std::max(base_fused_temp_bytes(ne), gsort_bytes);
      ba.temp = BUF(char, "g_sort_temp", ba.temp_bytes);
      return GS_OK;
    })());
    if (!any_base && gsort_bytes) {
      gs_status s2 = GS_OK;
      CHUNK_ALLOC(([&]() -> gs_status {
        ba.temp = buf<char>(ctx, "g_sort_temp", gsort_bytes, &s2);
        return ba.temp ? GS_OK : s2;
      })());
      ba.temp_bytes = gsort_bytes;
    }
#undef CHUNK_ALLOC
    for (int x = 1; x < 3 && use_fmm; ++x) {
      const int n = sg[x].n;
      if (n == 0) continue;
      hipLaunchKernelGGL(group_keys_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n,
                         wl.grp[x], nQ, gkey[x], gidx[x]);
      size_t bytes = ba.temp_bytes;
      DT_HIP(rocprim::radix_sort_pairs(ba.temp, bytes, gkey[x], const_cast<unsigned long long*>(sg[x].key),
                                       gidx[x], const_cast<int32_t*>(sg[x].order), (unsigned)n, 0, 64, st));
    }
    // The expansions write gdh, lco and pL only, the base cases gx only: the
    // expansions go to the side stream and overlap the base-case plan (whose
    // readbacks wait for the main stream alone) and tiles.  The side stream
    // is joined back when the chunk returns.  Pair logging keeps one stream:
    // its cost model is calibrated from the kernels' own times.
    struct SideJoin {
      hipStream_t st = nullptr, ss = nullptr;
      hipEvent_t ev = nullptr;
      ~SideJoin() {
        if (ss != st && (hipEventRecord(ev, ss) != hipSuccess || hipStreamWaitEvent(st, ev, 0) != hipSuccess))
          (void)hipGetLastError();
      }
    } join;
    join.st = join.ss = st;
    hipStream_t ss = st;
    if (use_fmm && !log_pairs && ctx->side) {
      DT_HIP(hipEventRecord(ctx->fork_ev, st));
      DT_HIP(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
      ss = join.ss = ctx->side;
      join.ev = ctx->join_ev;
    }
    if (use_fmm) {
      KernelTimer kt(ctx, ctx->kernel_timing, GS_K_SERIES, ss);
      {
        KernelTimer kd(ctx, ctx->kernel_timing, GS_K_DL, ss);
        if (fast)
          DT_HIP(launch_dl_fast(D, P, tensor, sg[1], wl.dl_slice, (int)used_slc[1], wl.dl_first, wl.dl_cpre,
                                wl.ent[1], qv, rv, xr_perm, wr_perm, d_sc, nQ, lco, pL, dl_part,
                                dl_part_p, ss));
        else
          DT_HIP(launch_dl(T, sg[1], wl.ent[1], qv, rv, xr_perm, wr_perm, d_sc, nQ, lco, pL, ss));
        kd.stop(ss, fast ? 2 : 1);
      }
      {
        KernelTimer kh(ctx, ctx->kernel_timing, GS_K_H2L, ss);
        if (fast) {
          DT_HIP(launch_h2l_fast(D, P, tensor, sg[2], wl.ent[2], qv, rv, Mom, d_sc, nQ, lco, pL, h2l_part,
                                 h2l_part_p, ss));
          kh.stop(ss, sg[2].n ? 2 : 0);
        } else {
          DT_HIP(launch_h2l(T, sg[2], wl.ent[2], qv, rv, Mom, d_sc, nQ, lco, pL, ss));
          kh.stop(ss, 1);
        }
      }
      KernelTimer kdh(ctx, ctx->kernel_timing, GS_K_DH, ss);
      int dh_launches = 0;
      for (size_t lv = 0; lv + 1 < dh_level_begin.size(); ++lv) {
        const int64_t gb = dh_level_begin[lv], ge = dh_level_begin[lv + 1];
        // query nodes of traversal level lv: nodes of depth lv, or leaves of
        // earlier levels (at most leaf_size points)
        const int depth_max = lv < qt.level_max.size() ? qt.level_max[lv] : 0;
        const int max_q = std::max(depth_max, opt.leaf_size);
        const int64_t sb = dh_slice_begin[lv], se = dh_slice_begin[lv + 1];
        if (ge == gb) continue;
        if (fast) {
          DT_HIP(launch_dh_fast(D, P, tensor, wl.dh_slice + sb, (int)(se - sb), (int)sb, wl.grp[0], wl.dh_first,
                                (int)gb, (int)(ge - gb), max_q, wl.ent[0], qv, rv, xq_perm, Mom, d_sc,
                                (int)Mq, gdh, dh_part, ss));
          dh_launches += se - sb > ge - gb ? 2 : 1;
        } else {
          DT_HIP(launch_dh_level(T, wl.grp[0] + gb, (int)(ge - gb), max_q, wl.ent[0], qv, rv, xq_perm,
                                 Mom, d_sc, (int)Mq, gdh, ss));
          dh_launches += 1;
        }
      }
      kdh.stop(ss, dh_launches);
      kt.stop(ss, (fast ? 3 : 2) + dh_launches);
    }
    if (any_base) {
      if (!rec_ready) {
        DT_HIP(launch_base_records(ra, st));
        rec_ready = true;
      }
      BaseFusedPlan plan;
      DT_HIP(plan_base_fused(ba, &plan, st));
      KernelTimer kt(ctx, ctx->kernel_timing, GS_K_BASE, st);
      DT_HIP(launch_base_fused(ba, plan, st));
      kt.stop(st, 1);
    }
    t_work += now_ms() - tb0;
    return GS_OK;
  };

  // 3-4. Traversal and work, over chunks of the bandwidth sweep.
  int chunk = opt.h_chunk > 0 ? std::min(opt.h_chunk, n_h) : n_h, h_chunks = 0;
  for (int hc0 = 0; hc0 < n_h;) {
    const int hc1 = std::min(n_h, hc0 + chunk);
    bool retry = false;
    s = run_chunk(hc0, hc1, &retry);
    if (s != GS_OK) return s;
    if (retry) {
      chunk = std::max(1, (hc1 - hc0) / 2);
      ctx->err.clear();
      continue;
    }
    ++h_chunks;
    hc0 = hc1;
  }
  double t4 = now_ms();
  S.t_traverse_ms = t_trav;
  S.t_work_ms = t_work;
  S.levels = max_level;
  S.frontier_peak = peak;
  S.h_chunks = h_chunks;

  // 5. Post-pass.
  KernelTimer kpost(ctx, ctx->kernel_timing, GS_K_POST, st);
  if (series_fast_available(D, P, tensor)) {
    DT_HIP(launch_leaf_post_fast(D, P, tensor, qv, qt.parent, nQ, n_h, (int)Mq, d_sc, xq_perm, qt.perm, gx, gdh,
                                 Gest, lco, pL, G_dev, st));
    kpost.stop(st, 1);
  } else {
    for (size_t lv = 0; lv + 1 < qt.level_begin.size(); ++lv)
      DT_HIP(launch_l2l_level(T, qv, qt.level_begin[lv], qt.level_begin[lv + 1], n_h, nQ, d_sc,
                              lco ? lco : Gest, pL, Gest, st));
    // one workgroup per query node; internal nodes exit at once
    DT_HIP(launch_leaf_eval(T, qv, nullptr, nQ, n_h, nQ, (int)Mq, d_sc, xq_perm, qt.perm, gx, gdh, Gest,
                            lco ? lco : Gest, pL, G_dev, st));
    kpost.stop(st, (int)qt.level_begin.size());
  }
  double t5 = now_ms();
  S.t_post_ms = t5 - t4;

  // Statistics: copied to pinned memory now, read after the call's final
  // synchronisation (finish_dualtree_stats).
  {
    hipError_t pe = hipSuccess;
    auto* hc = static_cast<unsigned long long*>(
        ctx->ws.get_pinned("stats_counts", sizeof(unsigned long long) * (n_h * 6 + kEvN), &pe));
    if (!hc) DT_FAIL(GS_ENOMEM, "pinned host allocation failed for the statistics");
    DT_HIP(hipMemcpyAsync(hc, hcount, sizeof(unsigned long long) * (n_h * 6 + kEvN), hipMemcpyDeviceToHost, st));
    ctx->stats_pending = hc;
    ctx->stats_pending_nh = n_h;
  }
  if (opt.keep_trace) {
    s = keep_tree(ctx, rt, D, ctx->host_tree[0], st);
    if (s != GS_OK) return s;
    s = keep_tree(ctx, qt, D, ctx->host_tree[1], st);
    if (s != GS_OK) return s;
  }
  if (log_pairs) {
    DT_HIP(hipStreamSynchronize(st));
    finish_dualtree_stats(ctx);
    flush_kernel_timers(ctx);
    policy_calibrate_costs(ctx, D);
    s = policy_build_records(ctx, D, hs);
    if (s != GS_OK) return s;
  }
  return GS_OK;
}

}  // namespace gs
