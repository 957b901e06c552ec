// Direct Hermite evaluation (DH) and direct local accumulation (DL) kernels
// specialised at compile time for the (dimension, order limit) pairs of the
// order-limit table (section 6), in double precision.
//
// With the multi-index set fixed at compile time (graded order, decreasing
// lexicographic inside a degree, built by a constexpr enumerator), the sums
// over multi-indices unroll completely: Hermite polynomial values stay in
// registers and every index into them is a constant.  Both kernels use
// h_a(t) = exp(-|t|^2) prod_d H_{a_d}(t_d), so one exponential serves all
// dimensions of a point.
//
//   DH:  gdh[h][q] += sum_{|a|<p} M_a s^{|a|} h_a((x_q - x_R) s)   (one wave per
//        slice of up to 8 entries of a group of a traversal level and per 64
//        points of Q, lanes over the points; the slices of a longer group
//        summed in order by a second kernel)
//   DL:  lco[h][Q][b] += sum_{r in R} w_r/b! h_b((x_r - x_Q) s)    (one wave per
//        slice of up to 16 chunks of 64 reference points, lanes over the
//        points, per-lane partial coefficients reduced across the wave once
//        per slice; then per (h, Q) run the slices summed in order)
//
// Every kernel also has an O(p^D) form (template flag T: tensor index sets,
// every a_d < p, ordered by largest component).  The nested sums then give
// each dimension the same bound p instead of the remaining degree, and the
// tensor DL uses the product form of its coefficients (dl_tensor_kernel).
#include "gs_series.h"

namespace gs {

namespace {

constexpr int kW = 64;
constexpr int kWavesPerBlock = 4;

constexpr int cbinom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long long c = 1;
  for (int i = 1; i <= k; ++i) c = c * (n - k + i) / i;
  return (int)c;
}

constexpr double cfact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

constexpr int cpow(int b, int e) {
  int v = 1;
  for (int i = 0; i < e; ++i) v *= b;
  return v;
}

// Multi-index set of order P in the library's order: graded (|a| < P, by
// degree, decreasing lexicographic inside a degree) or, with T, tensor
// (every a_d < P, by largest component, decreasing lexicographic inside).
// ord[i] < p tells whether term i belongs to order p; deg[i] = |a|.
template <int D, int P, bool T = false>
struct MultiIndex {
  static constexpr int C = T ? cpow(P, D) : cbinom(D + P - 1, D);
  int a[C][D];
  int deg[C];
  int ord[C];
  double invf[C];
  int nterms[P + 1];
  constexpr MultiIndex() : a(), deg(), ord(), invf(), nterms() {
    if (T) {
      int idx = 0;
      for (int m = 0; m < P; ++m) {
        const int n = cpow(m + 1, D);
        for (int k = 0; k < n; ++k) {
          // digits of k in base m + 1, most significant first, counted
          // down from m: decreasing lexicographic order
          int cur[D] = {};
          int r = k, mx = 0, sum = 0;
          for (int d = D - 1; d >= 0; --d) {
            cur[d] = m - r % (m + 1);
            r /= m + 1;
          }
          double f = 1.0;
          for (int d = 0; d < D; ++d) {
            mx = cur[d] > mx ? cur[d] : mx;
            sum += cur[d];
          }
          if (mx != m) continue;
          for (int d = 0; d < D; ++d) {
            a[idx][d] = cur[d];
            f *= cfact(cur[d]);
          }
          deg[idx] = sum;
          ord[idx] = m;
          invf[idx] = 1.0 / f;
          ++idx;
        }
      }
      for (int p = 0; p <= P; ++p) nterms[p] = cpow(p, D);
      return;
    }
    int idx = 0;
    for (int g = 0; g < P; ++g) {
      int cur[D] = {};
      cur[0] = g;
      while (true) {
        double f = 1.0;
        for (int d = 0; d < D; ++d) {
          a[idx][d] = cur[d];
          f *= cfact(cur[d]);
        }
        deg[idx] = g;
        ord[idx] = g;
        invf[idx] = 1.0 / f;
        ++idx;
        int i = D - 2;
        while (i >= 0 && cur[i] == 0) --i;
        if (i < 0) break;
        cur[i] -= 1;
        int rest = 1;
        for (int k = i + 1; k < D; ++k) {
          rest += cur[k];
          cur[k] = 0;
        }
        cur[i + 1] = rest;
      }
    }
    for (int p = 0; p <= P; ++p) nterms[p] = cbinom(D + p - 1, D);
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kW);
  return v;
}

// Physicists' Hermite polynomials H_0..H_{P-1}(t).
template <int P>
__device__ __forceinline__ void hermite_polys(double t, double* H) {
  H[0] = 1.0;
  if (P > 1) H[1] = 2.0 * t;
#pragma unroll
  for (int k = 1; k + 1 < P; ++k) H[k + 1] = 2.0 * t * H[k] - 2.0 * k * H[k - 1];
}

// Position of the multi-index (A...) in the set's order (compile time).
template <int D, int P, bool T, int... A>
constexpr int set_index() {
  constexpr MultiIndex<D, P, T> mi{};
  const int want[D] = {A...};
  for (int i = 0; i < MultiIndex<D, P, T>::C; ++i) {
    bool eq = true;
    for (int d = 0; d < D; ++d) eq = eq && mi.a[i][d] == want[d];
    if (eq) return i;
  }
  return -1;
}

// Nested (Horner-like) sum over the multi-indices of order p of
// M[a] prod_d H[d][a_d], dimension by dimension: each dimension's factor
// multiplies the sum over the dimensions after it, so a term costs one fused
// multiply-add instead of a product over all dimensions.  A... holds the
// indices of the dimensions before d; a runs over dimension d below rem: the
// remaining degree p - (a_0 + ... + a_{d-1}) of a graded set, or p itself in
// every dimension of a tensor set.
template <int D, int P, bool T, int d, int rem, int a, int... A>
struct DHNest {
  static __device__ __forceinline__ double run(const double (&H)[D][P], const double* __restrict__ M) {
    double inner;
    if constexpr (d == D - 1) {
      constexpr int I = set_index<D, P, T, A..., a>();
      static_assert(I >= 0, "multi-index outside the set");
      inner = M[I];
    } else {
      inner = DHNest<D, P, T, d + 1, T ? rem : rem - a, 0, A..., a>::run(H, M);
    }
    // (where H[d][0] is the constant 1 the compiler drops the product)
    const double v = H[d][a] * inner;
    if constexpr (a + 1 < rem)
      return v + DHNest<D, P, T, d, rem, a + 1, A...>::run(H, M);
    else
      return v;
  }
};

// The order p of an entry (1..P) selects the compile-time truncation.
template <int D, int P, bool T, int p = 1>
__device__ __forceinline__ double dh_sum(int pr, const double (&H)[D][P], const double* __restrict__ M) {
  if constexpr (p > P) {
    return 0.0;
  } else {
    if (pr == p) return DHNest<D, P, T, 0, p, 0>::run(H, M);
    return dh_sum<D, P, T, p + 1>(pr, H, M);
  }
}

// grid.x: slices of the level (kWavesPerBlock per block), grid.y: 64-point
// chunks of Q.
template <int D, int P, bool T>
__global__ __launch_bounds__(kW* kWavesPerBlock) void dh_fast_kernel(
    const int4* __restrict__ slc, int ns, const int4* __restrict__ grp,
    const int32_t* __restrict__ ent, NodeView qt, NodeView rt, const double* __restrict__ xq_perm,
    const double* __restrict__ M, const double* __restrict__ sc, int Mq, double* __restrict__ gdh,
    double* __restrict__ part) {
  constexpr int C = MultiIndex<D, P, T>::C;
  const int lane = threadIdx.x % kW;
  // wave index: uniform across the wave (readfirstlane tells the compiler)
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kW);
  if (i >= ns) return;
  const int4 sl = slc[i];
  const int4 gr = grp[sl.x];
  const int h = gr.x, Q = gr.y;
  const int qb = qt.begin[Q], qn = qt.count[Q];
  const int base = blockIdx.y * kW;
  if (base >= qn) return;
  const double s = sc[h];
  double spow[P];
  spow[0] = 1.0;
#pragma unroll
  for (int k = 1; k < P; ++k) spow[k] = spow[k - 1] * s;
  const bool active = base + lane < qn;
  const int qpos = qb + base + (active ? lane : 0);
  double x[D];
#pragma unroll
  for (int d = 0; d < D; ++d) x[d] = xq_perm[(int64_t)qpos * D + d];
  double acc = 0.0;
  for (int e = sl.y; e < sl.y + sl.z; ++e) {
    const int R = ent[e] >> 4, p = ent[e] & 15;
    const double* cR = rt.ctr + (int64_t)R * D;
    // H[d][k] = s^k H_k(t_d): the scale s^|a| of a term splits over the
    // dimensions
    double H[D][P];
    double tt = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double t = (x[d] - cR[d]) * s;
      tt += t * t;
      hermite_polys<P>(t, H[d]);
#pragma unroll
      for (int k = 1; k < P; ++k) H[d][k] *= spow[k];
    }
    const double v = dh_sum<D, P, T>(p, H, M + (int64_t)R * C);
    acc += v * exp(-tt);
  }
  if (!active) return;
  if (gr.w <= kDHSliceEntries)
    gdh[(int64_t)h * Mq + qpos] += acc;
  else
    part[((int64_t)i * gridDim.y + blockIdx.y) * kW + lane] = acc;
}

// Sum of a long DH group's slices, in slice order; grid as above over the
// level's groups.
__global__ __launch_bounds__(kW* kWavesPerBlock) void dh_reduce_kernel(
    const int4* __restrict__ grp, const int32_t* __restrict__ first, int g0, int ng, int slice0,
    NodeView qt, int Mq, const double* __restrict__ part, double* __restrict__ gdh) {
  const int lane = threadIdx.x % kW;
  // wave index: uniform across the wave (readfirstlane tells the compiler)
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kW);
  if (i >= ng) return;
  const int4 gr = grp[g0 + i];
  if (gr.w <= kDHSliceEntries) return;
  const int Q = gr.y, qn = qt.count[Q];
  const int base = blockIdx.y * kW;
  if (base + lane >= qn) return;
  const int ns = (gr.w + kDHSliceEntries - 1) / kDHSliceEntries;
  const int s0 = first[g0 + i] - slice0;
  double sum = 0.0;
  for (int k = 0; k < ns; ++k) sum += part[((int64_t)(s0 + k) * gridDim.y + blockIdx.y) * kW + lane];
  gdh[(int64_t)gr.x * Mq + qt.begin[Q] + base + lane] += sum;
}

// One wave per DL slice: lanes over 64 reference points of a chunk, per-lane
// partial coefficients reduced across the wave once per slice.
template <int D, int P>
__global__ __launch_bounds__(kW* kWavesPerBlock) void dl_fast_kernel(
    const int4* __restrict__ slc, int ns, const int4* __restrict__ grp,
    const int32_t* __restrict__ ent, const int32_t* __restrict__ cpre, NodeView qt, NodeView rt,
    const double* __restrict__ xr_perm, const double* __restrict__ wr_perm,
    const double* __restrict__ sc, double* __restrict__ part, int32_t* __restrict__ part_p) {
  constexpr MultiIndex<D, P> mi{};
  constexpr int C = MultiIndex<D, P>::C;
  const int lane = threadIdx.x % kW;
  // wave index: uniform across the wave (readfirstlane tells the compiler)
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kW);
  if (i >= ns) return;
  const int4 sl = slc[i];
  const int4 g0 = grp[sl.x];
  const int h = g0.x, Q = g0.y;
  const double s = sc[h];
  double cQ[D];
#pragma unroll
  for (int d = 0; d < D; ++d) cQ[d] = qt.ctr[(int64_t)Q * D + d];
  // entry holding the slice's first chunk: the last with cpre <= first chunk
  int lo = 0, hi = g0.w - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cpre[g0.z + mid] <= sl.y)
      lo = mid;
    else
      hi = mid - 1;
  }
  int e = g0.z + lo;
  int c = sl.y - cpre[e];  // chunk inside entry e
  double B[C];
#pragma unroll
  for (int a = 0; a < C; ++a) B[a] = 0.0;
  int pmax = 0;
  int R = ent[e] >> 4, p = ent[e] & 15;
  int rb = rt.begin[R], rn = rt.count[R];
  for (int k = sl.y; k < sl.z; ++k, ++c) {
    if (c * kW >= rn) {
      ++e;
      c = 0;
      R = ent[e] >> 4;
      p = ent[e] & 15;
      rb = rt.begin[R];
      rn = rt.count[R];
    }
    pmax = p > pmax ? p : pmax;
    if (c * kW + lane >= rn) continue;
    const int pos = rb + c * kW + lane;
    double H[D][P];
    double tt = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double t = (xr_perm[(int64_t)pos * D + d] - cQ[d]) * s;
      tt += t * t;
      hermite_polys<P>(t, H[d]);
    }
    const double ew = wr_perm[pos] * exp(-tt);
#pragma unroll
    for (int a = 0; a < C; ++a) {
      if (mi.ord[a] < p) {
        double term = ew;
#pragma unroll
        for (int d = 0; d < D; ++d)
          if (mi.a[a][d]) term *= H[d][mi.a[a][d]];
        B[a] += term;
      }
    }
  }
  double* out = part + (int64_t)i * C;
#pragma unroll
  for (int a = 0; a < C; ++a) {
    const double v = wave_sum(B[a]);
    if (lane == 0) out[a] = v;
  }
  if (lane == 0) part_p[i] = pmax;
}

// Position of each tensor multi-index in the set's order, by its dense
// row-major index sum_d a_d P^(D-1-d).
template <int D, int P>
struct TensorPos {
  int pos[cpow(P, D)];
  constexpr TensorPos() : pos() {
    constexpr MultiIndex<D, P, true> mi{};
    for (int i = 0; i < MultiIndex<D, P, true>::C; ++i) {
      int dense = 0;
      for (int d = 0; d < D; ++d) dense = dense * P + mi.a[i][d];
      pos[dense] = i;
    }
  }
};

// DL for tensor sets.  B_b = sum_r w_r e^{-|t_r|^2} prod_d H_{b_d}(t_rd) is a
// sum over the points of outer products, so a lane owns one combination of
// the trailing indices (b_1..b_{D-1}) and keeps the P values of b_0: per point
// one product over the trailing dimensions and P fused multiply-adds.  The
// points of a chunk are staged in LDS as u[r][d][k] = H_k(t_rd), times the
// point's w e^{-|t|^2} in dimension 0 and zero for k >= the entry's order, so
// that the terms outside an entry's order vanish.  With fewer combinations
// than lanes, G = 64 / NT lane groups split the points and are summed by a
// fixed butterfly at the end.  One wave per slice (the slices of
// dl_fast_kernel); part[slice][C] before the 1/b! scale, as dl_fast_kernel.
template <int D, int P>
__global__ __launch_bounds__(kW) void dl_tensor_kernel(
    const int4* __restrict__ slc, int ns, const int4* __restrict__ grp,
    const int32_t* __restrict__ ent, const int32_t* __restrict__ cpre, NodeView qt, NodeView rt,
    const double* __restrict__ xr_perm, const double* __restrict__ wr_perm,
    const double* __restrict__ sc, double* __restrict__ part, int32_t* __restrict__ part_p) {
  static constexpr TensorPos<D, P> tp{};
  constexpr int C = MultiIndex<D, P, true>::C;
  constexpr int NT = cpow(P, D - 1);                          // trailing combinations
  constexpr int G = (NT < kW && kW % NT == 0) ? kW / NT : 1;  // lane groups over points
  constexpr int NJ = G > 1 ? 1 : (NT + kW - 1) / kW;          // combinations per lane
  __shared__ double u[kW][D][P];
  const int lane = threadIdx.x;
  const int i = blockIdx.x;
  if (i >= ns) return;
  const int4 sl = slc[i];
  const int4 g0 = grp[sl.x];
  const int h = g0.x, Q = g0.y;
  const double s = sc[h];
  double cQ[D];
#pragma unroll
  for (int d = 0; d < D; ++d) cQ[d] = qt.ctr[(int64_t)Q * D + d];
  int lo = 0, hi = g0.w - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cpre[g0.z + mid] <= sl.y)
      lo = mid;
    else
      hi = mid - 1;
  }
  int e = g0.z + lo;
  int c = sl.y - cpre[e];
  // this lane's combinations and point group
  const int grpi = G > 1 ? lane / NT : 0;
  int combo[NJ], tb[NJ][D];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    combo[j] = G > 1 ? lane % NT : j * kW + lane;
    int r = combo[j] < NT ? combo[j] : 0;
#pragma unroll
    for (int d = D - 1; d >= 1; --d) {
      tb[j][d] = r % P;
      r /= P;
    }
    tb[j][0] = 0;
  }
  double B[NJ][P];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int k = 0; k < P; ++k) B[j][k] = 0.0;
  int pmax = 0;
  int R = ent[e] >> 4, p = ent[e] & 15;
  int rb = rt.begin[R], rn = rt.count[R];
  for (int k = sl.y; k < sl.z; ++k, ++c) {
    if (c * kW >= rn) {
      ++e;
      c = 0;
      R = ent[e] >> 4;
      p = ent[e] & 15;
      rb = rt.begin[R];
      rn = rt.count[R];
    }
    pmax = p > pmax ? p : pmax;
    const int cnt = rn - c * kW < kW ? rn - c * kW : kW;
    __syncthreads();  // the previous chunk's reads of u are done
    if (lane < cnt) {
      const int pos = rb + c * kW + lane;
      double H[D][P];
      double tt = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double t = (xr_perm[(int64_t)pos * D + d] - cQ[d]) * s;
        tt += t * t;
        hermite_polys<P>(t, H[d]);
      }
      const double ew = wr_perm[pos] * exp(-tt);
#pragma unroll
      for (int d = 0; d < D; ++d)
#pragma unroll
        for (int q = 0; q < P; ++q) u[lane][d][q] = q < p ? (d == 0 ? H[d][q] * ew : H[d][q]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if (combo[j] >= NT) continue;
      for (int r = grpi; r < cnt; r += G) {
        double t = 1.0;
#pragma unroll
        for (int d = 1; d < D; ++d) t *= u[r][d][tb[j][d]];
#pragma unroll
        for (int q = 0; q < P; ++q) B[j][q] += u[r][0][q] * t;
      }
    }
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int off = NT; off < kW; off <<= 1)
#pragma unroll
      for (int q = 0; q < P; ++q) B[0][q] += __shfl_xor(B[0][q], off, kW);
  }
  double* out = part + (int64_t)i * C;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    if (combo[j] >= NT || grpi != 0) continue;
#pragma unroll
    for (int q = 0; q < P; ++q) out[tp.pos[q * NT + combo[j]]] = B[j][q];
  }
  if (lane == 0) part_p[i] = pmax;
}

// Leaf moments (Figure 5, buildLeaf): M_a = sum_r w_r (x_r - x_R)^a / a!, one
// wave per node (internal nodes exit).  Graded sets: lanes over the points,
// per-lane partial moments reduced across the wave at the end.  Tensor sets:
// the product form of dl_tensor_kernel with powers in place of Hermite
// values (the moments are sums of outer products of per-dimension powers).
template <int D, int P>
__global__ __launch_bounds__(kW) void p2m_graded_kernel(NodeView t, int n_nodes, const double* __restrict__ xperm,
                                                        const double* __restrict__ wperm,
                                                        double* __restrict__ M) {
  static constexpr MultiIndex<D, P> mi{};
  constexpr int C = MultiIndex<D, P>::C;
  const int node = blockIdx.x;
  if (node >= n_nodes || t.left[node] >= 0) return;
  const int lane = threadIdx.x;
  const int b = t.begin[node], n = t.count[node];
  double c[D];
#pragma unroll
  for (int d = 0; d < D; ++d) c[d] = t.ctr[(int64_t)node * D + d];
  double B[C];
#pragma unroll
  for (int a = 0; a < C; ++a) B[a] = 0.0;
  for (int base = 0; base < n; base += kW) {
    if (base + lane >= n) continue;
    const int pos = b + base + lane;
    double U[D][P];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double u = xperm[(int64_t)pos * D + d] - c[d];
      U[d][0] = 1.0;
#pragma unroll
      for (int k = 1; k < P; ++k) U[d][k] = U[d][k - 1] * u;
    }
    const double w = wperm[pos];
#pragma unroll
    for (int a = 0; a < C; ++a) {
      double term = w;
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (mi.a[a][d]) term *= U[d][mi.a[a][d]];
      B[a] += term;
    }
  }
  double* out = M + (int64_t)node * C;
#pragma unroll
  for (int a = 0; a < C; ++a) {
    const double v = wave_sum(B[a]);
    if (lane == 0) out[a] = v * mi.invf[a];
  }
}

template <int D, int P>
__global__ __launch_bounds__(kW) void p2m_tensor_kernel(NodeView t, int n_nodes, const double* __restrict__ xperm,
                                                        const double* __restrict__ wperm,
                                                        double* __restrict__ M) {
  static constexpr MultiIndex<D, P, true> mi{};
  static constexpr TensorPos<D, P> tp{};
  constexpr int C = MultiIndex<D, P, true>::C;
  constexpr int NT = cpow(P, D - 1);
  constexpr int G = (NT < kW && kW % NT == 0) ? kW / NT : 1;
  constexpr int NJ = G > 1 ? 1 : (NT + kW - 1) / kW;
  __shared__ double u[kW][D][P];
  const int node = blockIdx.x;
  if (node >= n_nodes || t.left[node] >= 0) return;
  const int lane = threadIdx.x;
  const int b = t.begin[node], n = t.count[node];
  double c[D];
#pragma unroll
  for (int d = 0; d < D; ++d) c[d] = t.ctr[(int64_t)node * D + d];
  const int grpi = G > 1 ? lane / NT : 0;
  int combo[NJ], tb[NJ][D];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    combo[j] = G > 1 ? lane % NT : j * kW + lane;
    int r = combo[j] < NT ? combo[j] : 0;
#pragma unroll
    for (int d = D - 1; d >= 1; --d) {
      tb[j][d] = r % P;
      r /= P;
    }
    tb[j][0] = 0;
  }
  double B[NJ][P];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int k = 0; k < P; ++k) B[j][k] = 0.0;
  for (int base = 0; base < n; base += kW) {
    const int cnt = n - base < kW ? n - base : kW;
    __syncthreads();  // the previous chunk's reads of u are done
    if (lane < cnt) {
      const int pos = b + base + lane;
      const double w = wperm[pos];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double x = xperm[(int64_t)pos * D + d] - c[d];
        double v = d == 0 ? w : 1.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
          u[lane][d][k] = v;
          v *= x;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if (combo[j] >= NT) continue;
      for (int r = grpi; r < cnt; r += G) {
        double prod = 1.0;
#pragma unroll
        for (int d = 1; d < D; ++d) prod *= u[r][d][tb[j][d]];
#pragma unroll
        for (int q = 0; q < P; ++q) B[j][q] += u[r][0][q] * prod;
      }
    }
  }
  if constexpr (G > 1) {
#pragma unroll
    for (int off = NT; off < kW; off <<= 1)
#pragma unroll
      for (int q = 0; q < P; ++q) B[0][q] += __shfl_xor(B[0][q], off, kW);
  }
  double* out = M + (int64_t)node * C;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    if (combo[j] >= NT || grpi != 0) continue;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int i = tp.pos[q * NT + combo[j]];
      out[i] = B[j][q] * mi.invf[i];
    }
  }
}

// Position in the set's order of every multi-index of the dense box
// [0, P)^D (row-major), -1 outside the set.
template <int D, int P, bool T>
struct DensePos {
  int pos[cpow(P, D)];
  int dense[MultiIndex<D, P, T>::C];
  constexpr DensePos() : pos(), dense() {
    constexpr MultiIndex<D, P, T> mi{};
    for (int i = 0; i < cpow(P, D); ++i) pos[i] = -1;
    for (int i = 0; i < MultiIndex<D, P, T>::C; ++i) {
      int x = 0;
      for (int d = 0; d < D; ++d) x = x * P + mi.a[i][d];
      pos[x] = i;
      dense[i] = x;
    }
  }
};

// H2H (Lemma 2, raw moments) of the internal nodes [lb, le) of one level:
// M_g = sum over both children of sum_{a<=g} M'_a prod_d u_d^{g_d-a_d}/(g_d-a_d)!,
// u = x_child - x_node.  The translation is a product over dimensions, so it
// is applied as D one-dimensional passes (pass d replaces index d), each term
// costing at most P multiply-adds instead of the product over all a <= g.
// Both index families are closed under lowering a component, so every
// intermediate index stays in the set.  One wave per node, lanes over terms,
// the coefficient vector in LDS between passes.
template <int D, int P, bool T>
__global__ __launch_bounds__(kW) void h2h_fast_kernel(NodeView t, int lb, int le, double* __restrict__ M) {
  static constexpr MultiIndex<D, P, T> mi{};
  static constexpr DensePos<D, P, T> dp{};
  constexpr int C = MultiIndex<D, P, T>::C;
  constexpr int NB = (C + kW - 1) / kW;
  __shared__ double X[C];
  const int node = lb + blockIdx.x;
  if (node >= le) return;
  const int l = t.left[node];
  if (l < 0) return;
  const int lane = threadIdx.x;
  int stride[D];
  stride[D - 1] = 1;
#pragma unroll
  for (int d = D - 2; d >= 0; --d) stride[d] = stride[d + 1] * P;
  double acc[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) acc[u] = 0.0;
  for (int ch = 0; ch < 2; ++ch) {
    const int c = l + ch;
    double tr[D][P];  // u_d^m / m!
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double u = t.ctr[(int64_t)c * D + d] - t.ctr[(int64_t)node * D + d];
      tr[d][0] = 1.0;
#pragma unroll
      for (int m = 1; m < P; ++m) tr[d][m] = tr[d][m - 1] * u / (double)m;
    }
    __syncthreads();  // the previous child's reads of X are done
    for (int i = lane; i < C; i += kW) X[i] = M[(int64_t)c * C + i];
    __syncthreads();
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double y[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int i = u * kW + lane;
        y[u] = 0.0;
        if (i < C) {
          const int g = mi.a[i][d];
          const int base = dp.dense[i] - g * stride[d];
          for (int k = 0; k <= g; ++k) y[u] += tr[d][g - k] * X[dp.pos[base + k * stride[d]]];
        }
      }
      __syncthreads();  // every lane has read this pass's input
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (u * kW + lane < C) X[u * kW + lane] = y[u];
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (u * kW + lane < C) acc[u] += X[u * kW + lane];
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
    if (u * kW + lane < C) M[(int64_t)node * C + u * kW + lane] = acc[u];
}

// H2L (Lemma 1): B_b(Q) += (-1)^|b| / b! sum_{|a|<p} A_a h_{a+b}(t), t = (x_Q - x_R) s,
// one wave per H2L group (its entries in order), lanes over b.  Per entry the
// 1-D Hermite polynomials of orders < 2P-1 go to LDS; lane b forms
// g_d[k] = s^k H_{k+b_d}(t_d) (k < P) and the nested sum over a of
// M_a prod_d g_d[a_d] (M the raw moments, so A_a = M_a s^|a|), times
// exp(-|t|^2).  part[group][b] holds the group's sum before the 1/b! scale.
template <int D, int P, bool T>
__global__ __launch_bounds__(kW) void h2l_fast_kernel(
    const int4* __restrict__ grp, int ng, const int32_t* __restrict__ ent, NodeView qt, NodeView rt,
    const double* __restrict__ M, const double* __restrict__ sc, double* __restrict__ part,
    int32_t* __restrict__ part_p) {
  static constexpr MultiIndex<D, P, T> mi{};
  constexpr int C = MultiIndex<D, P, T>::C;
  constexpr int NB = (C + kW - 1) / kW;
  constexpr int HT = 2 * P - 1;
  __shared__ double Ht[D][HT];
  const int i = blockIdx.x;
  if (i >= ng) return;
  const int lane = threadIdx.x;
  const int4 gr = grp[i];
  const int h = gr.x, Q = gr.y;
  const double s = sc[h];
  double spow[P];
  spow[0] = 1.0;
#pragma unroll
  for (int k = 1; k < P; ++k) spow[k] = spow[k - 1] * s;
  int bd[NB][D], bdeg[NB], bord[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int b = u * kW + lane < C ? u * kW + lane : 0;
#pragma unroll
    for (int d = 0; d < D; ++d) bd[u][d] = mi.a[b][d];
    bdeg[u] = mi.deg[b];
    bord[u] = u * kW + lane < C ? mi.ord[b] : P;  // lanes past C never contribute
  }
  double acc[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) acc[u] = 0.0;
  int pmax = 0;
  const double* cQ = qt.ctr + (int64_t)Q * D;
  for (int e = gr.z; e < gr.z + gr.w; ++e) {
    const int R = ent[e] >> 4, p = ent[e] & 15;
    pmax = p > pmax ? p : pmax;
    const double* cR = rt.ctr + (int64_t)R * D;
    double tt = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double t = (cQ[d] - cR[d]) * s;
      tt += t * t;
    }
    __syncthreads();  // the previous entry's reads of Ht are done
    if (lane < D) {
      const double t = (cQ[lane] - cR[lane]) * s;
      double H[HT];
      hermite_polys<HT>(t, H);
#pragma unroll
      for (int k = 0; k < HT; ++k) Ht[lane][k] = H[k];
    }
    __syncthreads();
    const double ex = exp(-tt);
    const double* m = M + (int64_t)R * C;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      double g[D][P];
#pragma unroll
      for (int d = 0; d < D; ++d)
#pragma unroll
        for (int k = 0; k < P; ++k) g[d][k] = spow[k] * Ht[d][k + bd[u][d]];
      const double v = dh_sum<D, P, T>(p, g, m) * ex;
      if (bord[u] < p) acc[u] += (bdeg[u] & 1) ? -v : v;
    }
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
    if (u * kW + lane < C) part[(int64_t)i * C + u * kW + lane] = acc[u];
  if (lane == 0) part_p[i] = pmax;
}

// Per (h, Q) run of the sorted DL groups: the slices of its groups summed in
// order, scaled by 1/b! into lco; lanes over coefficients.  first == nullptr:
// one partial vector per group, at the group's index (H2L).
template <int D, int P, bool T>
__global__ __launch_bounds__(kW* kWavesPerBlock) void dl_reduce_kernel(
    SortedGroups g, const int2* __restrict__ first, const double* __restrict__ part,
    const int32_t* __restrict__ part_p, int nQ, double* __restrict__ lco, int32_t* __restrict__ pL) {
  static constexpr MultiIndex<D, P, T> mi{};
  constexpr int C = MultiIndex<D, P, T>::C;
  const int lane = threadIdx.x % kW;
  // wave index: uniform across the wave (readfirstlane tells the compiler)
  const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + threadIdx.x / kW);
  if (i >= g.n || (i > 0 && g.key[i] == g.key[i - 1])) return;
  const int4 g0 = g.grp[g.order[i]];
  const int h = g0.x, Q = g0.y;
  double sum[(C + kW - 1) / kW];
#pragma unroll
  for (int u = 0; u < (C + kW - 1) / kW; ++u) sum[u] = 0.0;
  int pmax = 0;
  for (int j = i; j < g.n && (j == i || g.key[j] == g.key[j - 1]); ++j) {
    const int2 f = first ? first[g.order[j]] : make_int2(g.order[j], 1);
    for (int k = f.x; k < f.x + f.y; ++k) {
      const double* v = part + (int64_t)k * C;
#pragma unroll
      for (int u = 0; u < (C + kW - 1) / kW; ++u)
        if (u * kW + lane < C) sum[u] += v[u * kW + lane];
      pmax = part_p[k] > pmax ? part_p[k] : pmax;
    }
  }
  double* out = lco + ((int64_t)h * nQ + Q) * C;
#pragma unroll
  for (int u = 0; u < (C + kW - 1) / kW; ++u) {
    const int a = u * kW + lane;
    if (a < C) out[a] += sum[u] * mi.invf[a];
  }
  if (lane == 0) {
    int32_t* pl = pL + (int64_t)h * nQ + Q;
    *pl = pmax > *pl ? pmax : *pl;
  }
}

// Post-pass (Figure 8) of one query leaf and one bandwidth, without the
// level-by-level translation: the result at a point adds, over the leaf and
// its ancestors A, Gest_A and A's own local expansion evaluated at the point.
// A local-to-local translation re-expands a polynomial exactly, so this is
// the same sum as translating every expansion down to the leaf first.
template <int D, int P, bool T>
__global__ __launch_bounds__(kW) void leaf_post_kernel(
    NodeView qt, const int32_t* __restrict__ parent, int nQ, int Mq, const double* __restrict__ sc,
    const double* __restrict__ xq_perm, const int32_t* __restrict__ qperm,
    const double* __restrict__ gx, const double* __restrict__ gdh, const double* __restrict__ Gest,
    const double* __restrict__ lco, const int32_t* __restrict__ pL, double* __restrict__ G_out) {
  constexpr int C = MultiIndex<D, P, T>::C;
  const int Q = blockIdx.x;
  const int h = blockIdx.y;
  if (Q >= nQ || qt.left[Q] >= 0) return;
  const int lane = threadIdx.x;
  const int64_t hb = (int64_t)h * nQ;
  double ge = 0.0;  // finite-difference sums, from the leaf up
  for (int A = Q; A >= 0; A = parent[A]) ge += Gest[hb + A];
  const double s = sc[h];
  const int qb = qt.begin[Q], qn = qt.count[Q];
  for (int base = 0; base < qn; base += kW) {
    const bool active = base + lane < qn;
    const int qpos = qb + base + (active ? lane : 0);
    double x[D];
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = xq_perm[(int64_t)qpos * D + d];
    double v = gx[(int64_t)h * Mq + qpos] + gdh[(int64_t)h * Mq + qpos] + ge;
    for (int A = Q; A >= 0; A = parent[A]) {
      const int p = pL[hb + A];
      if (p == 0) continue;
      const double* cA = qt.ctr + (int64_t)A * D;
      double U[D][P];  // powers of (x - c_A) s
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double u = (x[d] - cA[d]) * s;
        U[d][0] = 1.0;
#pragma unroll
        for (int k = 1; k < P; ++k) U[d][k] = U[d][k - 1] * u;
      }
      v += dh_sum<D, P, T>(p, U, lco + (hb + A) * C);
    }
    if (active) G_out[(int64_t)h * Mq + qperm[qpos]] = v;
  }
}

template <int D, int P, bool T>
void dh_launch(const int4* slices, int ns, int slice0, const int4* grp, const int32_t* first, int g0,
               int ng, int max_q, const int32_t* ent, const NodeView& qt, const NodeView& rt,
               const double* xq, const double* M, const double* sc, int Mq, double* gdh, double* part,
               hipStream_t s) {
  const unsigned cy = (unsigned)ceil_div(max_q, kW);
  hipLaunchKernelGGL((dh_fast_kernel<D, P, T>), dim3((unsigned)ceil_div(ns, kWavesPerBlock), cy),
                     dim3(kW * kWavesPerBlock), 0, s, slices, ns, grp, ent, qt, rt, xq, M, sc, Mq, gdh,
                     part);
  if (ng > 0 && ns > ng)  // some group has more than one slice
    hipLaunchKernelGGL(dh_reduce_kernel, dim3((unsigned)ceil_div(ng, kWavesPerBlock), cy),
                       dim3(kW * kWavesPerBlock), 0, s, grp, first, g0, ng, slice0, qt, Mq, part, gdh);
}

template <int D, int P, bool T>
void dl_launch(const SortedGroups& g, const int4* slices, int ns, const int2* first,
               const int32_t* cpre, const int32_t* ent, const NodeView& qt, const NodeView& rt,
               const double* xr, const double* wr, const double* sc, int nQ, double* lco, int32_t* pL,
               double* part, int32_t* part_p, hipStream_t s) {
  if constexpr (T)
    hipLaunchKernelGGL((dl_tensor_kernel<D, P>), dim3((unsigned)ns), dim3(kW), 0, s, slices, ns, g.grp,
                       ent, cpre, qt, rt, xr, wr, sc, part, part_p);
  else
    hipLaunchKernelGGL((dl_fast_kernel<D, P>), dim3((unsigned)ceil_div(ns, kWavesPerBlock)),
                       dim3(kW * kWavesPerBlock), 0, s, slices, ns, g.grp, ent, cpre, qt, rt, xr, wr, sc,
                       part, part_p);
  hipLaunchKernelGGL((dl_reduce_kernel<D, P, T>), dim3((unsigned)ceil_div(g.n, kWavesPerBlock)),
                     dim3(kW * kWavesPerBlock), 0, s, g, first, part, part_p, nQ, lco, pL);
}

template <int D, int P, bool T>
void h2h_launch(const NodeView& t, int lb, int le, double* M, hipStream_t s) {
  hipLaunchKernelGGL((h2h_fast_kernel<D, P, T>), dim3((unsigned)(le - lb)), dim3(kW), 0, s, t, lb, le, M);
}

template <int D, int P, bool T>
void p2m_launch(const NodeView& t, int n_nodes, const double* xperm, const double* wperm, double* M,
                hipStream_t s) {
  if constexpr (T)
    hipLaunchKernelGGL((p2m_tensor_kernel<D, P>), dim3((unsigned)n_nodes), dim3(kW), 0, s, t, n_nodes, xperm,
                       wperm, M);
  else
    hipLaunchKernelGGL((p2m_graded_kernel<D, P>), dim3((unsigned)n_nodes), dim3(kW), 0, s, t, n_nodes, xperm,
                       wperm, M);
}

// (D, P) pairs with a compiled specialisation: graded sets at the order
// limits of section 6, tensor sets at the O(p^D) limits (in one dimension,
// and at order 1, the two sets coincide and the graded kernels serve both).
#define GS_FAST_CASES(X) \
  X(1, 10, false) X(2, 8, false) X(3, 6, false) X(4, 5, false) X(5, 4, false) X(6, 2, false) \
  X(7, 1, false) X(8, 1, false) X(16, 1, false) \
  X(2, 8, true) X(3, 6, true) X(4, 4, true) X(5, 3, true) X(6, 2, true)

// The set family a (D, P, tensor) request runs with.
bool tensor_kernels(int D, int P, bool tensor) { return tensor && D > 1 && P > 1; }

}  // namespace

bool series_fast_available(int D, int P, bool tensor) {
  const bool t = tensor_kernels(D, P, tensor);
#define X(d, p, tt) \
  if (D == d && P == p && t == tt) return true;
  GS_FAST_CASES(X)
#undef X
  return false;
}

hipError_t launch_dh_fast(int D, int P, bool tensor, const int4* slices, int ns, int slice0, const int4* grp,
                          const int32_t* first, int g0, int ng, int max_q, const int32_t* ent,
                          const NodeView& qt, const NodeView& rt, const double* xq_perm,
                          const double* M, const double* sc, int Mq, double* gdh, double* part,
                          hipStream_t s) {
  if (ns == 0) return hipSuccess;
  const bool t = tensor_kernels(D, P, tensor);
#define X(d, p, tt)                                                                                 \
  if (D == d && P == p && t == tt) {                                                                \
    dh_launch<d, p, tt>(slices, ns, slice0, grp, first, g0, ng, max_q, ent, qt, rt, xq_perm, M, sc, \
                        Mq, gdh, part, s);                                                          \
    return hipGetLastError();                                                                       \
  }
  GS_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_dl_fast(int D, int P, bool tensor, const SortedGroups& g, const int4* slices, int ns,
                          const int2* first, const int32_t* cpre, const int32_t* ent,
                          const NodeView& qt, const NodeView& rt, const double* xr_perm,
                          const double* wr_perm, const double* sc, int nQ, double* lco, int32_t* pL,
                          double* part, int32_t* part_p, hipStream_t s) {
  if (g.n == 0 || ns == 0) return hipSuccess;
  const bool t = tensor_kernels(D, P, tensor);
#define X(d, p, tt)                                                                                   \
  if (D == d && P == p && t == tt) {                                                                  \
    dl_launch<d, p, tt>(g, slices, ns, first, cpre, ent, qt, rt, xr_perm, wr_perm, sc, nQ, lco, pL,   \
                        part, part_p, s);                                                             \
    return hipGetLastError();                                                                         \
  }
  GS_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

int series_terms(int D, int P, bool tensor) { return tensor ? cpow(P, D) : cbinom(D + P - 1, D); }

hipError_t launch_h2l_fast(int D, int P, bool tensor, const SortedGroups& g, const int32_t* ent,
                           const NodeView& qt, const NodeView& rt, const double* M, const double* sc,
                           int nQ, double* lco, int32_t* pL, double* part, int32_t* part_p,
                           hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const bool t = tensor_kernels(D, P, tensor);
#define X(d, p, tt)                                                                                    \
  if (D == d && P == p && t == tt) {                                                                   \
    hipLaunchKernelGGL((h2l_fast_kernel<d, p, tt>), dim3((unsigned)g.n), dim3(kW), 0, s, g.grp, g.n,    \
                       ent, qt, rt, M, sc, part, part_p);                                              \
    hipLaunchKernelGGL((dl_reduce_kernel<d, p, tt>), dim3((unsigned)ceil_div(g.n, kWavesPerBlock)),    \
                       dim3(kW * kWavesPerBlock), 0, s, g, (const int2*)nullptr, part, part_p, nQ,     \
                       lco, pL);                                                                       \
    return hipGetLastError();                                                                          \
  }
  GS_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_h2h_level_fast(int D, int P, bool tensor, const NodeView& t, int lb, int le, double* M,
                                 hipStream_t s) {
  if (le <= lb) return hipSuccess;
  const bool tk = tensor_kernels(D, P, tensor);
#define X(d, p, tt)                                   \
  if (D == d && P == p && tk == tt) {                 \
    h2h_launch<d, p, tt>(t, lb, le, M, s);            \
    return hipGetLastError();                         \
  }
  GS_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_p2m_fast(int D, int P, bool tensor, const NodeView& t, int n_nodes, const double* xperm,
                           const double* wperm, double* M, hipStream_t s) {
  const bool tk = tensor_kernels(D, P, tensor);
#define X(d, p, tt)                                                       \
  if (D == d && P == p && tk == tt) {                                     \
    p2m_launch<d, p, tt>(t, n_nodes, xperm, wperm, M, s);                 \
    return hipGetLastError();                                             \
  }
  GS_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_leaf_post_fast(int D, int P, bool tensor, const NodeView& qt, const int32_t* parent, int nQ,
                                 int n_h, int Mq, const double* sc, const double* xq_perm,
                                 const int32_t* qperm, const double* gx, const double* gdh,
                                 const double* Gest, const double* lco, const int32_t* pL,
                                 double* G_out, hipStream_t s) {
  const bool t = tensor_kernels(D, P, tensor);
#define X(d, p, tt)                                                                                  \
  if (D == d && P == p && t == tt) {                                                                 \
    hipLaunchKernelGGL((leaf_post_kernel<d, p, tt>), dim3((unsigned)nQ, (unsigned)n_h), dim3(kW), 0,  \
                       s, qt, parent, nQ, Mq, sc, xq_perm, qperm, gx, gdh, Gest, lco, pL, G_out);    \
    return hipGetLastError();                                                                        \
  }
  GS_FAST_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace gs
