// kd-tree construction on the GPU (section 6, Figure 5).
//
// Split rule (the paper leaves it open): a node with more than leaf_size
// points is split on its dimension of widest bounding-box extent (ties to the
// smallest dimension); its points ordered by (coordinate, original index)
// go to the left child for the first left_count(n) = half of n rounded up to a
// multiple of leaf_size, and to the right child for the rest.  Every node
// whose count is a multiple of leaf_size then splits into two such nodes, so
// all leaves but one hold exactly leaf_size points: whole waves of 64 lanes
// for the kernels that put one point per lane.  Nodes are numbered breadth
// first, left before right.
//
// Construction without per-level sorting: each dimension d keeps a list of
// point ids sorted by (x_d, id) inside every node's position range
// [begin, begin+count) (one stable radix sort per dimension at the start), plus
// one extra list sorted by id.  A node's bounding box is then read off the
// first and last entry of each list, and its split assigns the first
// left_count(n) entries of the split dimension's list to the left child.  Every
// list is then stably partitioned by that assignment (one exclusive scan of
// the per-entry flags over all lists at once), which keeps each list sorted
// inside both children.  The extra list becomes the final permutation, whose
// leaves hold their points in increasing original index.
//
// All values cached per node are exact or computed in a fixed order:
// lo/hi are copies of coordinates, ctr = 0.5*(lo+hi), rinf = max over points of
// |x - ctr|_inf, which equals max_d max(|lo_d - ctr_d|, |hi_d - ctr_d|) and is
// read off the box; leaf W is the sequential sum in permutation order,
// internal W = W_left + W_right.
#include <cstring>  // rocprim uses memset without including it
#include <rocprim/rocprim.hpp>

#include <algorithm>

#include "gs_internal.h"
#include "gs_tree.h"

namespace gs {

namespace {

__device__ __forceinline__ int64_t left_count(int64_t n, int leaf_size) {
  return (int64_t)leaf_size * ((n + 2 * (int64_t)leaf_size - 1) / (2 * (int64_t)leaf_size));
}

__global__ void iota_kernel(int32_t* __restrict__ v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int32_t)i;
}

__global__ void node_stats_kernel(int lb, int le, int D, int64_t n, const int32_t* __restrict__ lists,
                                  const double* __restrict__ xs, const int32_t* __restrict__ begin,
                                  const int32_t* __restrict__ count, double* __restrict__ lo,
                                  double* __restrict__ hi, double* __restrict__ ctr,
                                  int32_t* __restrict__ splitdim, double* __restrict__ rinf) {
  const int i = lb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= le) return;
  const int64_t b = begin[i];
  const int64_t c = count[i];
  int best = 0;
  double bestext = -1.0;
  double r = 0.0;
  for (int d = 0; d < D; ++d) {
    const double l = xs[(int64_t)d * n + lists[(int64_t)d * n + b]];
    const double h = xs[(int64_t)d * n + lists[(int64_t)d * n + b + c - 1]];
    const double m = 0.5 * (l + h);
    lo[(int64_t)i * D + d] = l;
    hi[(int64_t)i * D + d] = h;
    ctr[(int64_t)i * D + d] = m;
    const double ext = h - l;
    if (ext > bestext) {
      bestext = ext;
      best = d;
    }
    // max over the node's points of |x_d - m| is attained at x_d = lo or hi
    const double a = fabs(l - m), e = fabs(h - m);
    r = a > r ? a : r;
    r = e > r ? e : r;
  }
  splitdim[i] = best;
  rinf[i] = r;
}

// Per position of the level: left/right assignment and next-level node.
__global__ void mark_kernel(int64_t n, int leaf_size, const int32_t* __restrict__ lists,
                            const int32_t* __restrict__ pos_node,
                            int32_t* __restrict__ pos_node_next, int32_t* __restrict__ leaf_of_pos,
                            const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
                            const int32_t* __restrict__ left, const int32_t* __restrict__ splitdim,
                            int32_t* __restrict__ isleft) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int node = pos_node[i];
  if (node < 0) {
    pos_node_next[i] = -1;
    return;
  }
  const int l = left[node];
  if (l >= 0) {
    const int64_t mid = (int64_t)begin[node] + left_count(count[node], leaf_size);
    const int sd = splitdim[node];
    isleft[lists[(int64_t)sd * n + i]] = i < mid ? 1 : 0;
    pos_node_next[i] = i < mid ? l : l + 1;
  } else {
    leaf_of_pos[i] = node;
    pos_node_next[i] = -1;
  }
}

__global__ void flags_kernel(int64_t n, int nl, const int32_t* __restrict__ lists,
                             const int32_t* __restrict__ pos_node, const int32_t* __restrict__ left,
                             const int32_t* __restrict__ isleft, int32_t* __restrict__ flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nl) return;
  const int64_t i = t % n;
  const int node = pos_node[i];
  flags[t] = (node >= 0 && left[node] >= 0) ? isleft[lists[t]] : 0;
}

__global__ void scatter_kernel(int64_t n, int nl, int leaf_size, const int32_t* __restrict__ lists,
                               const int32_t* __restrict__ pos_node, const int32_t* __restrict__ left,
                               const int32_t* __restrict__ begin, const int32_t* __restrict__ count,
                               const int32_t* __restrict__ flags, const int32_t* __restrict__ scan,
                               int32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nl) return;
  const int64_t k = t / n;
  const int64_t i = t - k * n;
  const int node = pos_node[i];
  int64_t dst = i;
  if (node >= 0 && left[node] >= 0) {
    const int64_t b = begin[node];
    const int64_t half = left_count(count[node], leaf_size);
    const int64_t rank = (int64_t)scan[t] - (int64_t)scan[k * n + b];
    dst = flags[t] ? b + rank : b + half + (i - b - rank);
  }
  out[k * n + dst] = lists[t];
}

// One wave per node (leaves only): the lanes load 64 weights at a time, the
// sum is taken in point order (one lane's value after another), the minimum
// by a wave reduction.
__global__ __launch_bounds__(256) void leaf_weights_kernel(int n_nodes, const int32_t* __restrict__ left,
                                                           const int32_t* __restrict__ begin,
                                                           const int32_t* __restrict__ count,
                                                           const int32_t* __restrict__ perm,
                                                           const double* __restrict__ w,
                                                           double* __restrict__ W,
                                                           double* __restrict__ wmin) {
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (int)(threadIdx.x / 64));
  const int lane = threadIdx.x % 64;
  if (i >= n_nodes || left[i] >= 0) return;
  double s = 0.0, m = INFINITY;
  const int b = begin[i], n = count[i];
  for (int c = 0; c < n; c += 64) {
    const int k = n - c < 64 ? n - c : 64;
    const double v = lane < k ? (w ? w[perm[b + c + lane]] : 1.0) : INFINITY;
    m = v < m ? v : m;
    for (int j = 0; j < k; ++j) {
      const long long bits = __double_as_longlong(v);
      const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), j);
      const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), j);
      s = s + __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = o < m ? o : m;
  }
  if (lane == 0) {
    W[i] = s;
    wmin[i] = m;
  }
}

__global__ void internal_weights_kernel(int lb, int le, const int32_t* __restrict__ left,
                                        double* __restrict__ W, double* __restrict__ wmin) {
  const int i = lb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= le) return;
  const int l = left[i];
  if (l < 0) return;
  W[i] = W[l] + W[l + 1];
  wmin[i] = wmin[l] < wmin[l + 1] ? wmin[l] : wmin[l + 1];
}

// One block per node: the largest squared distance of the node's points to
// its box centre (squares summed in d order), then its square root.
__global__ __launch_bounds__(256) void node_radius_kernel(const int32_t* __restrict__ begin,
                                                          const int32_t* __restrict__ count,
                                                          const double* __restrict__ ctr,
                                                          const double* __restrict__ x, int D,
                                                          double* __restrict__ rad) {
  __shared__ double part[4];
  const int i = blockIdx.x;
  const int64_t b = begin[i], c = count[i];
  const double* ci = ctr + (int64_t)i * D;
  double m = 0.0;
  for (int64_t k = threadIdx.x; k < c; k += blockDim.x) {
    const double* xp = x + (b + k) * D;
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
      const double diff = xp[d] - ci[d];
      s = s + diff * diff;
    }
    m = s > m ? s : m;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) m = part[w] > m ? part[w] : m;
    rad[i] = sqrt(m);
  }
}

}  // namespace

hipError_t launch_node_radius(const DevTree& t, int64_t n_nodes, const double* x_perm, int D,
                              hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(node_radius_kernel, dim3((unsigned)n_nodes), dim3(256), 0, s, t.begin, t.count,
                     t.ctr, x_perm, D, t.rad);
  return hipGetLastError();
}

int64_t tree_node_capacity(int64_t n, int leaf_size) {
  int64_t min_leaf = (leaf_size + 1) / 2;
  if (min_leaf < 1) min_leaf = 1;
  return 2 * (n / min_leaf + 1) + 1;
}

size_t tree_sort_temp_bytes(int64_t n, int D) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs((void*)nullptr, bytes, (const double*)nullptr, (double*)nullptr,
                            (const int32_t*)nullptr, (int32_t*)nullptr, (unsigned)n);
  size_t b2 = 0;
  (void)rocprim::exclusive_scan((void*)nullptr, b2, (const int32_t*)nullptr, (int32_t*)nullptr, 0,
                          (size_t)n * (D + 1), rocprim::plus<int32_t>());
  return bytes > b2 ? bytes : b2;
}

hipError_t build_tree_device(const TreeBuildArgs& a, DevTree& t, std::vector<int>& level_begin,
                             hipStream_t s) {
  const int64_t n = a.n;
  const int D = a.D;
  const int nl = D + 1;
  hipError_t e;
  const unsigned g1 = (unsigned)ceil_div(n, 256);
  const unsigned gl = (unsigned)ceil_div(n * nl, 256);

  // Per-dimension lists sorted by (x_d, id), plus the id list.
  hipLaunchKernelGGL(iota_kernel, dim3(g1), dim3(256), 0, s, a.ids, n);
  for (int d = 0; d < D; ++d) {
    size_t bytes = a.temp_bytes;
    e = rocprim::radix_sort_pairs(a.temp, bytes, a.xs + (int64_t)d * n, a.sort_keys, a.ids,
                                  a.lists + (int64_t)d * n, (unsigned)n, 0, 64, s);
    if (e != hipSuccess) return e;
  }
  e = hipMemcpyAsync(a.lists + (int64_t)D * n, a.ids, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;

  // Topology on the host (the counts depend on n and leaf_size only), in
  // breadth-first numbering, uploaded from pinned memory without a wait.
  const int64_t cap = t.capacity;
  int32_t* hb = a.host_topo;
  int32_t* hc = hb + cap;
  int32_t* hl = hc + cap;
  int32_t* hd = hl + cap;
  int32_t* hp = hd + cap;
  hb[0] = 0;
  hc[0] = (int32_t)n;
  hd[0] = 0;
  hp[0] = -1;
  int64_t nn = 1;
  level_begin.clear();
  int lb = 0, le = 1;
  while (true) {
    level_begin.push_back(lb);
    const int64_t before = nn;
    for (int i = lb; i < le; ++i) {
      if (hc[i] > a.leaf_size) {
        if (nn + 2 > cap) return hipErrorInvalidValue;
        const int64_t lc = (int64_t)a.leaf_size * ((hc[i] + 2 * (int64_t)a.leaf_size - 1) / (2 * (int64_t)a.leaf_size));
        hl[i] = (int32_t)nn;
        hb[nn] = hb[i];
        hc[nn] = (int32_t)lc;
        hb[nn + 1] = hb[i] + (int32_t)lc;
        hc[nn + 1] = hc[i] - (int32_t)lc;
        hd[nn] = hd[nn + 1] = hd[i] + 1;
        hp[nn] = hp[nn + 1] = i;
        nn += 2;
      } else {
        hl[i] = -1;
      }
    }
    if (nn == before) break;
    lb = le;
    le = (int)nn;
  }
  t.level_max.assign(level_begin.size(), 0);
  for (size_t lv = 0; lv < level_begin.size(); ++lv) {
    const int e0 = lv + 1 < level_begin.size() ? level_begin[lv + 1] : (int)nn;
    for (int i = level_begin[lv]; i < e0; ++i) t.level_max[lv] = std::max(t.level_max[lv], hc[i]);
  }
  e = hipMemcpyAsync(t.begin, hb, nn * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(t.count, hc, nn * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(t.left, hl, nn * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(t.depth, hd, nn * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(t.parent, hp, nn * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(a.pos_node, 0, n * sizeof(int32_t), s);
  if (e != hipSuccess) return e;

  int32_t* lists = a.lists;
  int32_t* lists_alt = a.lists_alt;
  int32_t* pos = a.pos_node;
  int32_t* pos_alt = a.pos_node_alt;
  for (size_t lv = 0; lv + 1 < level_begin.size() || lv + 1 == level_begin.size(); ++lv) {
    const int b0 = level_begin[lv];
    const int e0 = lv + 1 < level_begin.size() ? level_begin[lv + 1] : (int)nn;
    const int width = e0 - b0;
    hipLaunchKernelGGL(node_stats_kernel, dim3((unsigned)ceil_div(width, 256)), dim3(256), 0, s, b0,
                       e0, D, n, lists, a.xs, t.begin, t.count, t.lo, t.hi, t.ctr, a.splitdim,
                       t.rinf);
    hipLaunchKernelGGL(mark_kernel, dim3(g1), dim3(256), 0, s, n, a.leaf_size, lists, pos, pos_alt,
                       t.leaf_of_pos, t.begin, t.count, t.left, a.splitdim, a.isleft);
    if (lv + 1 == level_begin.size()) break;  // the last level has no children
    hipLaunchKernelGGL(flags_kernel, dim3(gl), dim3(256), 0, s, n, nl, lists, pos, t.left, a.isleft,
                       a.flags);
    size_t bytes = a.temp_bytes;
    e = rocprim::exclusive_scan(a.temp, bytes, a.flags, a.scan, 0, (size_t)n * nl,
                                rocprim::plus<int32_t>(), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scatter_kernel, dim3(gl), dim3(256), 0, s, n, nl, a.leaf_size, lists, pos, t.left, t.begin,
                       t.count, a.flags, a.scan, lists_alt);
    std::swap(lists, lists_alt);
    std::swap(pos, pos_alt);
  }
  le = (int)nn;
  level_begin.push_back(le);
  t.n_nodes = le;
  t.n_points = n;
  t.D = D;
  t.perm_list = lists + (int64_t)D * n;
  e = hipMemcpyAsync(t.perm, t.perm_list, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(leaf_weights_kernel, dim3((unsigned)ceil_div(le, 4)), dim3(256), 0, s, le,
                     t.left, t.begin, t.count, t.perm, a.w, t.W, t.wmin);
  for (int lv = (int)level_begin.size() - 2; lv >= 0; --lv) {
    const int b = level_begin[lv], en = level_begin[lv + 1];
    hipLaunchKernelGGL(internal_weights_kernel, dim3((unsigned)ceil_div(en - b, 256)), dim3(256), 0,
                       s, b, en, t.left, t.W, t.wmin);
  }
  return hipGetLastError();
}

}  // namespace gs
