// Hermite and Taylor expansion kernels (sections 1-3, Lemmas 1-3; Figures 5,
// 7 and 8), in double precision.
//
// With s = 1/sqrt(2h^2):
//   raw moments   M_a   = sum_r w_r (x_r - x_R)^a / a!            (buildLeaf)
//   H2H           M_g   = sum_{a<=g} M'_a (x_R' - x_R)^{g-a}/(g-a)!   (Lemma 2, raw form)
//   far field     sum_{|a|<p} M_a s^{|a|} h_a((x_q - x_R) s)      (EVALM / direct Hermite)
//   local (DL)    B_b  += sum_r w_r/b! h_b((x_r - x_Q) s)           (DIRECTL)
//   local (H2L)   B_b  += (-1)^{|b|}/b! sum_a M_a s^{|a|} h_{a+b}((x_Q - x_R) s)  (Lemma 1)
//   L2L           C_a   = sum_{b>=a} b!/(a!(b-a)!) B_b ((x_Q - x_Q') s)^{b-a}       (Lemma 3)
//   EVALL         sum_{|b|<p} B_b ((x_q - x_Q) s)^b
// with h_n(t) = exp(-t^2) H_n(t) from H_{n+1} = 2t H_n - 2n H_{n-1}.
//
// Work lists are processed one workgroup (one wave) per run of groups that
// share a (bandwidth, query node) key; the groups were sorted by key, stably,
// so a run lists its groups in traversal order and each output location is
// written by exactly one wave, in a fixed order: the results are deterministic.
#include "gs_series.h"

namespace gs {

namespace {

constexpr int kW = 64;  // one wave per workgroup
constexpr int kAccPerLane = (kMaxTerms + kW - 1) / kW;

// Hermite functions h_0..h_{n-1}(t) into out[0..n-1] (stride 1).
__device__ __forceinline__ void hermite_fns(double t, int n, double* out) {
  if (n <= 0) return;
  const double e = exp(-t * t);
  double hm1 = 1.0, h0 = 2.0 * t;  // H_0, H_1
  out[0] = e;
  if (n > 1) out[1] = h0 * e;
  for (int k = 1; k + 1 < n; ++k) {
    const double hn = 2.0 * t * h0 - 2.0 * k * hm1;
    hm1 = h0;
    h0 = hn;
    out[k + 1] = hn * e;
  }
}

// True for the first sorted group of a run (a new (h, Q) key).
__device__ __forceinline__ bool run_start(const SortedGroups& g, int i) {
  return i == 0 || g.key[i] != g.key[i - 1];
}

// ---------------------------------------------------------------- moments

__global__ __launch_bounds__(kW) void p2m_kernel(SeriesTables T, NodeView t, int n_nodes,
                                                 const double* __restrict__ xperm,
                                                 const double* __restrict__ wperm,
                                                 double* __restrict__ M) {
  extern __shared__ double lds[];
  const int node = blockIdx.x;
  if (node >= n_nodes || t.left[node] >= 0) return;
  const int D = T.D, P = T.P, C = T.C;
  double* pw = lds;                 // [kW][D][P]
  double* wl = lds + kW * D * P;    // [kW]
  const int b = t.begin[node], n = t.count[node];
  const double* c = t.ctr + (int64_t)node * D;
  double acc[kAccPerLane];
  for (int k = 0; k < kAccPerLane; ++k) acc[k] = 0.0;
  for (int base = 0; base < n; base += kW) {
    const int cnt = n - base < kW ? n - base : kW;
    const int lane = threadIdx.x;
    if (lane < cnt) {
      const int pos = b + base + lane;
      for (int d = 0; d < D; ++d) {
        const double u = xperm[(int64_t)pos * D + d] - c[d];
        double v = 1.0;
        for (int k = 0; k < P; ++k) {
          pw[(lane * D + d) * P + k] = v;
          v *= u;
        }
      }
      wl[lane] = wperm[pos];
    }
    __syncthreads();
    for (int a = lane, ai = 0; a < C; a += kW, ++ai) {
      const int8_t* al = T.alpha + a * D;
      double s = 0.0;
      for (int r = 0; r < cnt; ++r) {
        double m = wl[r];
        for (int d = 0; d < D; ++d) m *= pw[(r * D + d) * P + al[d]];
        s += m;
      }
      acc[ai] += s;
    }
    __syncthreads();
  }
  for (int a = threadIdx.x, ai = 0; a < C; a += kW, ++ai)
    M[(int64_t)node * C + a] = acc[ai] * T.inv_fact[a];
}

__global__ __launch_bounds__(kW) void h2h_kernel(SeriesTables T, NodeView t, int lb, int le,
                                                 double* __restrict__ M) {
  extern __shared__ double lds[];
  const int node = lb + blockIdx.x;
  if (node >= le) return;
  const int l = t.left[node];
  if (l < 0) return;
  const int D = T.D, C = T.C;
  double* mono = lds;  // [2][C]: (x_child - x_node)^delta / delta!
  for (int ch = 0; ch < 2; ++ch) {
    const double* cc = t.ctr + (int64_t)(l + ch) * D;
    const double* cp = t.ctr + (int64_t)node * D;
    for (int dl = threadIdx.x; dl < C; dl += kW) {
      const int8_t* al = T.alpha + dl * D;
      double m = T.inv_fact[dl];
      for (int d = 0; d < D; ++d) {
        const double u = cc[d] - cp[d];
        for (int k = 0; k < al[d]; ++k) m *= u;
      }
      mono[ch * C + dl] = m;
    }
  }
  __syncthreads();
  for (int gm = threadIdx.x; gm < C; gm += kW) {
    double total = 0.0;
    for (int ch = 0; ch < 2; ++ch) {
      const double* Mc = M + (int64_t)(l + ch) * C;
      double s = 0.0;
      for (int k = T.h2h_start[gm]; k < T.h2h_start[gm + 1]; ++k) {
        const int2 pr = T.h2h_pairs[k];
        s += Mc[pr.x] * mono[ch * C + pr.y];
      }
      total = ch == 0 ? s : total + s;
    }
    M[(int64_t)node * C + gm] = total;
  }
}

// ------------------------------------------------------- direct Hermite (DH)
// DH pairs change per-point sums, and query nodes of different traversal
// levels overlap (an ancestor and its descendant), so DH work is launched once
// per traversal level, in level order: inside one level the query nodes of a
// bandwidth are disjoint, hence each wave owns its points' gdh entries.

__global__ __launch_bounds__(kW) void dh_kernel(SeriesTables T, const int4* __restrict__ grp, int ng,
                                                const int32_t* __restrict__ ent, NodeView qt,
                                                NodeView rt, const double* __restrict__ xq_perm,
                                                const double* __restrict__ M,
                                                const double* __restrict__ sc, int Mq,
                                                double* __restrict__ gdh) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  if (i >= ng) return;
  const int D = T.D, P = T.P, C = T.C;
  double* Hq = lds;                 // [kW][D][P]
  double* A = lds + kW * D * P;     // [C]
  const int4 gr = grp[i];
  const int h = gr.x, Q = gr.y;
  const double s = sc[h];
  const int qb = qt.begin[Q], qn = qt.count[Q];
  const int lane = threadIdx.x;
  {
    const int base = blockIdx.y * kW;
    if (base >= qn) return;
    const bool active = base + lane < qn;
    const int qpos = qb + base + (active ? lane : 0);
    double acc = 0.0;
    for (int e = gr.z; e < gr.z + gr.w; ++e) {
      const int R = ent[e] >> 4, p = ent[e] & 15;
      const int nt = T.nterms[p];
      const double* cR = rt.ctr + (int64_t)R * D;
      for (int a = lane; a < nt; a += kW) {
        double sp = 1.0;
        for (int k = 0; k < T.deg[a]; ++k) sp *= s;
        A[a] = M[(int64_t)R * C + a] * sp;
      }
      for (int d = 0; d < D; ++d)
        hermite_fns((xq_perm[(int64_t)qpos * D + d] - cR[d]) * s, p, Hq + (lane * D + d) * P);
      __syncthreads();
      double v = 0.0;
      for (int a = 0; a < nt; ++a) {
        const int8_t* al = T.alpha + a * D;
        double m = A[a];
        for (int d = 0; d < D; ++d) m *= Hq[(lane * D + d) * P + al[d]];
        v += m;
      }
      acc += v;
      __syncthreads();
    }
    if (active) gdh[(int64_t)h * Mq + qpos] += acc;
  }
}

// ----------------------------------------------------- direct local (DL)

__global__ __launch_bounds__(kW) void dl_kernel(SeriesTables T, SortedGroups g,
                                                const int32_t* __restrict__ ent, NodeView qt,
                                                NodeView rt, const double* __restrict__ xr_perm,
                                                const double* __restrict__ wr_perm,
                                                const double* __restrict__ sc, int nQ,
                                                double* __restrict__ lco, int32_t* __restrict__ pL) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  if (i >= g.n || !run_start(g, i)) return;
  const int D = T.D, P = T.P, C = T.C;
  double* Hr = lds;               // [kW][D][P]
  double* wl = lds + kW * D * P;  // [kW]
  const int4 g0 = g.grp[g.order[i]];
  const int h = g0.x, Q = g0.y;
  const double s = sc[h];
  const double* cQ = qt.ctr + (int64_t)Q * D;
  const int lane = threadIdx.x;
  double acc[kAccPerLane];
  for (int k = 0; k < kAccPerLane; ++k) acc[k] = 0.0;
  int pmax = 0;
  for (int j = i; j < g.n && (j == i || !run_start(g, j)); ++j) {
    const int4 gr = g.grp[g.order[j]];
    for (int e = gr.z; e < gr.z + gr.w; ++e) {
      const int R = ent[e] >> 4, p = ent[e] & 15;
      pmax = p > pmax ? p : pmax;
      const int nt = T.nterms[p];
      const int rb = rt.begin[R], rn = rt.count[R];
      for (int base = 0; base < rn; base += kW) {
        const int cnt = rn - base < kW ? rn - base : kW;
        if (lane < cnt) {
          const int pos = rb + base + lane;
          for (int d = 0; d < D; ++d)
            hermite_fns((xr_perm[(int64_t)pos * D + d] - cQ[d]) * s, p, Hr + (lane * D + d) * P);
          wl[lane] = wr_perm[pos];
        }
        __syncthreads();
        for (int b = lane, bi = 0; b < nt; b += kW, ++bi) {
          const int8_t* al = T.alpha + b * D;
          double v = 0.0;
          for (int r = 0; r < cnt; ++r) {
            double m = wl[r];
            for (int d = 0; d < D; ++d) m *= Hr[(r * D + d) * P + al[d]];
            v += m;
          }
          acc[bi] += v;
        }
        __syncthreads();
      }
    }
  }
  double* out = lco + ((int64_t)h * nQ + Q) * C;
  for (int b = lane, bi = 0; b < C; b += kW, ++bi) out[b] += acc[bi] * T.inv_fact[b];
  if (lane == 0) {
    int32_t* pl = pL + (int64_t)h * nQ + Q;
    *pl = pmax > *pl ? pmax : *pl;
  }
}

// ------------------------------------------------------------------- H2L

__global__ __launch_bounds__(kW) void h2l_kernel(SeriesTables T, SortedGroups g,
                                                 const int32_t* __restrict__ ent, NodeView qt,
                                                 NodeView rt, const double* __restrict__ M,
                                                 const double* __restrict__ sc, int nQ,
                                                 double* __restrict__ lco, int32_t* __restrict__ pL) {
  extern __shared__ double lds[];
  const int i = blockIdx.x;
  if (i >= g.n || !run_start(g, i)) return;
  const int D = T.D, P = T.P, C = T.C;
  const int HT = 2 * P - 1;        // orders 0 .. 2P-2
  double* Ht = lds;                // [D][HT]
  double* A = lds + D * HT;        // [C]
  const int4 g0 = g.grp[g.order[i]];
  const int h = g0.x, Q = g0.y;
  const double s = sc[h];
  const double* cQ = qt.ctr + (int64_t)Q * D;
  const int lane = threadIdx.x;
  double acc[kAccPerLane];
  for (int k = 0; k < kAccPerLane; ++k) acc[k] = 0.0;
  int pmax = 0;
  for (int j = i; j < g.n && (j == i || !run_start(g, j)); ++j) {
    const int4 gr = g.grp[g.order[j]];
    for (int e = gr.z; e < gr.z + gr.w; ++e) {
      const int R = ent[e] >> 4, p = ent[e] & 15;
      pmax = p > pmax ? p : pmax;
      const int nt = T.nterms[p];
      const double* cR = rt.ctr + (int64_t)R * D;
      for (int d = lane; d < D; d += kW) hermite_fns((cQ[d] - cR[d]) * s, 2 * p - 1, Ht + d * HT);
      for (int a = lane; a < nt; a += kW) {
        double sp = 1.0;
        for (int k = 0; k < T.deg[a]; ++k) sp *= s;
        A[a] = M[(int64_t)R * C + a] * sp;
      }
      __syncthreads();
      for (int b = lane, bi = 0; b < nt; b += kW, ++bi) {
        const int8_t* bl = T.alpha + b * D;
        double v = 0.0;
        for (int a = 0; a < nt; ++a) {
          const int8_t* al = T.alpha + a * D;
          double m = A[a];
          for (int d = 0; d < D; ++d) m *= Ht[d * HT + al[d] + bl[d]];
          v += m;
        }
        acc[bi] += (T.deg[b] & 1) ? -v : v;
      }
      __syncthreads();
    }
  }
  double* out = lco + ((int64_t)h * nQ + Q) * C;
  for (int b = lane, bi = 0; b < C; b += kW, ++bi) out[b] += acc[bi] * T.inv_fact[b];
  if (lane == 0) {
    int32_t* pl = pL + (int64_t)h * nQ + Q;
    *pl = pmax > *pl ? pmax : *pl;
  }
}

// ----------------------------------------------------- post-pass (Figure 8)

__global__ __launch_bounds__(kW) void l2l_kernel(SeriesTables T, NodeView qt, int lb, int le, int nQ,
                                                 const double* __restrict__ sc,
                                                 double* __restrict__ lco, int32_t* __restrict__ pL,
                                                 double* __restrict__ Gest) {
  extern __shared__ double lds[];
  const int node = lb + blockIdx.x;
  const int h = blockIdx.y;
  if (node >= le) return;
  const int l = qt.left[node];
  if (l < 0) return;
  const int D = T.D, C = T.C;
  const int64_t me = (int64_t)h * nQ + node;
  const int p = pL[me];
  const double s = sc[h];
  double* mono = lds;  // [C]
  for (int ch = 0; ch < 2; ++ch) {
    const int c = l + ch;
    const int64_t ce = (int64_t)h * nQ + c;
    if (threadIdx.x == 0) Gest[ce] += Gest[me];
    if (p == 0) continue;
    const int nt = T.nterms[p];
    const double* cc = qt.ctr + (int64_t)c * D;
    const double* cp = qt.ctr + (int64_t)node * D;
    for (int g = threadIdx.x; g < nt; g += kW) {
      const int8_t* al = T.alpha + g * D;
      double m = 1.0;
      for (int d = 0; d < D; ++d) {
        const double u = (cc[d] - cp[d]) * s;
        for (int k = 0; k < al[d]; ++k) m *= u;
      }
      mono[g] = m;
    }
    __syncthreads();
    const double* B = lco + me * C;
    double* out = lco + ce * C;
    for (int a = threadIdx.x; a < nt; a += kW) {
      double v = 0.0;
      for (int k = T.l2l_start[a]; k < T.l2l_start[a + 1]; ++k) {
        const int2 pr = T.l2l_pairs[k];
        if (pr.x >= nt) break;
        v += T.l2l_coef[k] * B[pr.x] * mono[pr.y];
      }
      out[a] += v;
    }
    if (threadIdx.x == 0) pL[ce] = p > pL[ce] ? p : pL[ce];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kW) void leaf_eval_kernel(SeriesTables T, NodeView qt,
                                                       const int32_t* __restrict__ leaves,
                                                       int n_leaves, int nQ, int Mq,
                                                       const double* __restrict__ sc,
                                                       const double* __restrict__ xq_perm,
                                                       const int32_t* __restrict__ qperm,
                                                       const double* __restrict__ gx,
                                                       const double* __restrict__ gdh,
                                                       const double* __restrict__ Gest,
                                                       const double* __restrict__ lco,
                                                       const int32_t* __restrict__ pL,
                                                       double* __restrict__ G_out) {
  extern __shared__ double lds[];
  const int li = blockIdx.x;
  const int h = blockIdx.y;
  if (li >= n_leaves) return;
  // leaves == nullptr: one workgroup per node, internal nodes exit
  const int Q = leaves ? leaves[li] : li;
  if (!leaves && qt.left[Q] >= 0) return;
  const int D = T.D, P = T.P, C = T.C;
  const int64_t me = (int64_t)h * nQ + Q;
  const int p = pL[me];
  const int nt = p > 0 ? T.nterms[p] : 0;
  const double ge = Gest[me];
  const double s = sc[h];
  const double* B = lco + me * C;
  const double* cQ = qt.ctr + (int64_t)Q * D;
  double* pw = lds;  // [kW][D][P]
  const int qb = qt.begin[Q], qn = qt.count[Q];
  const int lane = threadIdx.x;
  for (int base = 0; base < qn; base += kW) {
    if (base + lane >= qn) continue;
    const int qpos = qb + base + lane;
    double v = gx[(int64_t)h * Mq + qpos] + gdh[(int64_t)h * Mq + qpos] + ge;
    if (nt > 0) {
      for (int d = 0; d < D; ++d) {
        const double u = (xq_perm[(int64_t)qpos * D + d] - cQ[d]) * s;
        double x = 1.0;
        for (int k = 0; k < P; ++k) {
          pw[(lane * D + d) * P + k] = x;
          x *= u;
        }
      }
      double e = 0.0;
      for (int b = 0; b < nt; ++b) {
        const int8_t* bl = T.alpha + b * D;
        double m = B[b];
        for (int d = 0; d < D; ++d) m *= pw[(lane * D + d) * P + bl[d]];
        e += m;
      }
      v += e;
    }
    G_out[(int64_t)h * Mq + qperm[qpos]] = v;
  }
}

}  // namespace

hipError_t launch_p2m(const SeriesTables& T, const NodeView& t, int n_nodes, const double* xperm,
                      const double* wperm, double* M, hipStream_t s) {
  const size_t lds = (size_t)(kW * T.D * T.P + kW) * sizeof(double);
  hipLaunchKernelGGL(p2m_kernel, dim3(n_nodes), dim3(kW), lds, s, T, t, n_nodes, xperm, wperm, M);
  return hipGetLastError();
}

hipError_t launch_h2h_level(const SeriesTables& T, const NodeView& t, int lb, int le, double* M,
                            hipStream_t s) {
  if (le <= lb) return hipSuccess;
  hipLaunchKernelGGL(h2h_kernel, dim3(le - lb), dim3(kW), (size_t)2 * T.C * sizeof(double), s, T, t,
                     lb, le, M);
  return hipGetLastError();
}

hipError_t launch_dh_level(const SeriesTables& T, const int4* grp, int ng, int max_q,
                           const int32_t* ent, const NodeView& qt, const NodeView& rt,
                           const double* xq_perm, const double* M, const double* sc, int Mq,
                           double* gdh, hipStream_t s) {
  if (ng == 0) return hipSuccess;
  const size_t lds = (size_t)(kW * T.D * T.P + T.C) * sizeof(double);
  hipLaunchKernelGGL(dh_kernel, dim3(ng, (unsigned)ceil_div(max_q, kW)), dim3(kW), lds, s, T, grp, ng,
                     ent, qt, rt, xq_perm, M, sc, Mq, gdh);
  return hipGetLastError();
}

hipError_t launch_dl(const SeriesTables& T, const SortedGroups& g, const int32_t* ent,
                     const NodeView& qt, const NodeView& rt, const double* xr_perm,
                     const double* wr_perm, const double* sc, int nQ, double* lco, int32_t* pL,
                     hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const size_t lds = (size_t)(kW * T.D * T.P + kW) * sizeof(double);
  hipLaunchKernelGGL(dl_kernel, dim3(g.n), dim3(kW), lds, s, T, g, ent, qt, rt, xr_perm, wr_perm, sc,
                     nQ, lco, pL);
  return hipGetLastError();
}

hipError_t launch_h2l(const SeriesTables& T, const SortedGroups& g, const int32_t* ent,
                      const NodeView& qt, const NodeView& rt, const double* M, const double* sc,
                      int nQ, double* lco, int32_t* pL, hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  const size_t lds = (size_t)(T.D * (2 * T.P - 1) + T.C) * sizeof(double);
  hipLaunchKernelGGL(h2l_kernel, dim3(g.n), dim3(kW), lds, s, T, g, ent, qt, rt, M, sc, nQ, lco, pL);
  return hipGetLastError();
}

hipError_t launch_l2l_level(const SeriesTables& T, const NodeView& qt, int lb, int le, int n_h,
                            int nQ, const double* sc, double* lco, int32_t* pL, double* Gest,
                            hipStream_t s) {
  if (le <= lb) return hipSuccess;
  hipLaunchKernelGGL(l2l_kernel, dim3(le - lb, n_h), dim3(kW), (size_t)T.C * sizeof(double), s, T,
                     qt, lb, le, nQ, sc, lco, pL, Gest);
  return hipGetLastError();
}

hipError_t launch_leaf_eval(const SeriesTables& T, const NodeView& qt, const int32_t* leaves,
                            int n_leaves, int n_h, int nQ, int Mq, const double* sc,
                            const double* xq_perm, const int32_t* qperm, const double* gx,
                            const double* gdh, const double* Gest, const double* lco,
                            const int32_t* pL, double* G_out, hipStream_t s) {
  const size_t lds = (size_t)kW * T.D * T.P * sizeof(double);
  hipLaunchKernelGGL(leaf_eval_kernel, dim3(n_leaves, n_h), dim3(kW), lds, s, T, qt, leaves,
                     n_leaves, nQ, Mq, sc, xq_perm, qperm, gx, gdh, Gest, lco, pL, G_out);
  return hipGetLastError();
}

}  // namespace gs
