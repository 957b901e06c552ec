// Frontier decision and emission kernels of the level-synchronous dual-tree
// traversal (sections 5-6, Figures 6-7).
//
// The frontier of a level is a list of segments; a segment is one bandwidth h
// and one query node Q with the reference nodes R_1..R_k still to be handled
// against Q, in left-to-right tree order.  One thread handles one segment,
// sequentially, because the token rule of section 5 makes each decision depend
// on the budget left by the previous ones:
//
//   L = Lpush_Q + sum_j W_Rj K(dmax(Q,R_j))   (and >= wmin_Q when the queries are
//                                               the references: the self term)
//   for each R_j:  FD if need(E_FD) <= t (finite difference);
//                  else bestMethod at maxerr = eps (W_R + t) L / W (Figure 6);
//                  else base case if both are leaves, else split.
//   need(E) = W E / (eps L) - W_R is the token a pruning costs; it is
//   subtracted from t (a negative need is a deposit).
//
// Every value that takes part in a decision is a double computed with
// separately rounded IEEE operations in a fixed order (this file is compiled
// without floating-point contraction) and with the exponential below, so the
// decisions are reproducible bit for bit by any implementation of the same
// arithmetic.
//
// The emission kernel then turns the per-pair decisions into the next
// frontier (children pairs in the same left-to-right order) and appends the
// resolved pairs to typed work lists, grouped per segment.
#include <cstring>  // rocprim uses memset without including it
#include <rocprim/rocprim.hpp>

#include "gs_traverse.h"

namespace gs {

namespace {

// exp(x) by Cody-Waite reduction and a degree-13 Taylor polynomial:
// x = k ln2 + r with k = floor(x log2(e) + 1/2), r = (x - k LN2_HI) - k LN2_LO
// (LN2_HI has enough trailing zero bits for k LN2_HI to be exact), exp(x) =
// 2^k P(r), P by Horner's rule.  Arguments below -700 give 0.
__device__ __forceinline__ double own_exp(double x) {
  constexpr double kLog2e = 1.4426950408889634;
  constexpr double kLn2Hi = 6.93147180369123816490e-01;
  constexpr double kLn2Lo = 1.90821492927058770002e-10;
  constexpr double c[14] = {1.0,
                            1.0,
                            1.0 / 2.0,
                            1.0 / 6.0,
                            1.0 / 24.0,
                            1.0 / 120.0,
                            1.0 / 720.0,
                            1.0 / 5040.0,
                            1.0 / 40320.0,
                            1.0 / 362880.0,
                            1.0 / 3628800.0,
                            1.0 / 39916800.0,
                            1.0 / 479001600.0,
                            1.0 / 6227020800.0};
  if (x < -700.0) return 0.0;
  const double k = floor(x * kLog2e + 0.5);
  const double r = (x - k * kLn2Hi) - k * kLn2Lo;
  double p = c[13];
#pragma unroll
  for (int n = 12; n >= 0; --n) p = p * r + c[n];
  return ldexp(p, (int)k);
}

__device__ __forceinline__ double powi(double x, int p) {
  double v = 1.0;
  for (int i = 0; i < p; ++i) v = v * x;
  return v;
}

constexpr int64_t kInfCost = INT64_MAX;

__device__ __forceinline__ int64_t sat_mul(int64_t a, int64_t b) {
  int64_t v;
  if (__builtin_mul_overflow(a, b, &v)) return kInfCost;
  return v < kInfCost ? v : kInfCost;
}

__device__ __forceinline__ int64_t pow_int(int64_t D, int e) {
  int64_t v = 1;
  for (int i = 0; i < e; ++i) v = sat_mul(v, D);
  return v;
}

__device__ __forceinline__ double need_fn(double E, double WR, double L, double W, double eps) {
  if (E == 0.0) return -WR;
  if (L == 0.0) return INFINITY;
  return (W * E) / (eps * L) - WR;
}

// Figure 6: smallest feasible order per method, then the cheapest by the
// cost model, first minimum in the order DH, DL, H2L, DIRECT.
__device__ void best_method(const DecideConst& c, double maxerr, double WR, double g, double rQ,
                            double rR, int64_t NQ, int64_t NR, int* code, int* p_out, double* E_out) {
  constexpr double kSqrt2 = 1.4142135623730951;
  int pf[3] = {0, 0, 0};
  double Ef[3] = {0.0, 0.0, 0.0};
  for (int p = 1; p <= c.P && (c.fmm_mask & 1); ++p) {
    const double E = ((WR * g) * c.bconst[p]) * powi(rR, p);
    if (E <= maxerr) {
      pf[0] = p;
      Ef[0] = E;
      break;
    }
  }
  for (int p = 1; p <= c.P && (c.fmm_mask & 2); ++p) {
    const double E = ((WR * g) * c.bconst[p]) * powi(rQ, p);
    if (E <= maxerr) {
      pf[1] = p;
      Ef[1] = E;
      break;
    }
  }
  for (int p = 1; p <= c.P && (c.fmm_mask & 4); ++p) {
    const double sq = kSqrt2 * rQ;
    const double itail = sq <= 1.0 ? 1.0 : powi(sq, p - 1);
    const double second = (powi(kSqrt2 * rR, p) * c.binomD[p]) * itail;
    const double E = ((WR * g) * c.bconst[p]) * (powi(rQ, p) + second);
    if (E <= maxerr) {
      pf[2] = p;
      Ef[2] = E;
      break;
    }
  }
  int64_t cost[4];
  cost[0] = pf[0] ? sat_mul(NQ, pow_int(c.D, pf[0] + 1)) : kInfCost;
  cost[1] = pf[1] ? sat_mul(NR, pow_int(c.D, pf[1] + 1)) : kInfCost;
  cost[2] = pf[2] ? pow_int(c.D, 2 * pf[2] + 1) : kInfCost;
  cost[3] = sat_mul(c.D, sat_mul(NQ, NR));
  int64_t best = cost[0];
  for (int i = 1; i < 4; ++i) best = cost[i] < best ? cost[i] : best;
  for (int i = 0; i < 3; ++i) {
    if (cost[i] == best && pf[i]) {
      *code = DH + i;
      *p_out = pf[i];
      *E_out = Ef[i];
      return;
    }
  }
  *code = -1;
  *p_out = 0;
  *E_out = INFINITY;
}

__device__ __forceinline__ void box_dist2(const double* loQ, const double* hiQ, const double* loR,
                                          const double* hiR, int D, double* dmin2, double* dmax2) {
  double smin = 0.0, smax = 0.0;
  for (int d = 0; d < D; ++d) {
    double gap = loQ[d] - hiR[d];
    double other = loR[d] - hiQ[d];
    if (other > gap) gap = other;
    if (gap < 0.0) gap = 0.0;
    double far = hiQ[d] - loR[d];
    other = hiR[d] - loQ[d];
    if (other > far) far = other;
    smin = smin + gap * gap;
    smax = smax + far * far;
  }
  *dmin2 = smin;
  *dmax2 = smax;
}

__global__ void decide_kernel(int S, FrontierLevel cur, TreeView qt, TreeView rt,
                              const double* __restrict__ inv2h2, const double* __restrict__ inv4h2,
                              const double* __restrict__ invh, int nQ, DecideConst c,
                              double* __restrict__ s_kmax, double* __restrict__ s_dmin2,
                              int8_t* __restrict__ code_out, int8_t* __restrict__ p_out,
                              double* __restrict__ Gest, SegCount* __restrict__ cnt,
                              unsigned long long* __restrict__ hcount,
                              unsigned long long* __restrict__ base_evals) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int h = cur.h[s];
  const int Q = cur.Q[s];
  const int off = cur.off[s];
  const int len = cur.len[s];
  double t = cur.T[s];
  double Lp = cur.Lp[s];
  const int D = c.D;
  const double* loQ = qt.lo + (int64_t)Q * D;
  const double* hiQ = qt.hi + (int64_t)Q * D;
  const double i2 = inv2h2[h], i4 = inv4h2[h], ih = invh[h];
  const bool qleaf = qt.left[Q] < 0;
  const int64_t NQ = qt.count[Q];

  // Lower bound on G over Q.
  double L = Lp;
  for (int j = 0; j < len; ++j) {
    const int R = cur.R[off + j];
    double dmin2, dmax2;
    box_dist2(loQ, hiQ, rt.lo + (int64_t)R * D, rt.hi + (int64_t)R * D, D, &dmin2, &dmax2);
    const double km = own_exp(-dmax2 * i2);
    s_kmax[off + j] = km;
    s_dmin2[off + j] = dmin2;
    L = L + rt.W[R] * km;
  }
  if (c.mono && qt.wmin[Q] > L) L = qt.wmin[Q];

  SegCount sc;
  for (int k = 0; k < 10; ++k) sc.v[k] = 0;
  int nchild = 0;
  double gest = 0.0;
  bool any_fd = false;
  int counts[6] = {0, 0, 0, 0, 0, 0};
  int64_t bevals = 0;
  for (int j = 0; j < len; ++j) {
    const int R = cur.R[off + j];
    const double WR = rt.W[R];
    const double km = s_kmax[off + j];
    const double dmin2 = s_dmin2[off + j];
    const double kmin = own_exp(-dmin2 * i2);
    const double efd = 0.5 * (WR * (kmin - km));
    const double nd = need_fn(efd, WR, L, c.Wtot, c.eps_alg);
    int cd = -1, p = 0;
    if (nd <= (c.use_tokens ? t : 0.0)) {
      if (c.use_tokens) t = t - nd;
      if (!any_fd) {
        gest = Gest[(int64_t)h * nQ + Q];
        any_fd = true;
      }
      gest = gest + 0.5 * (WR * (kmin + km));
      cd = FD;
    } else if (c.use_fmm) {
      const double tt = c.use_tokens ? t : 0.0;
      const double maxerr = ((c.eps_alg * (WR + tt)) * L) / c.Wtot;
      const double g = own_exp(-dmin2 * i4);
      double E;
      best_method(c, maxerr, WR, g, qt.rinf[Q] * ih, rt.rinf[R] * ih, NQ, rt.count[R], &cd, &p, &E);
      if (cd >= 0) {
        if (c.use_tokens) t = t - need_fn(E, WR, L, c.Wtot, c.eps_alg);
      } else {
        p = 0;
      }
    }
    const bool rleaf = rt.left[R] < 0;
    if (cd < 0) {
      if (qleaf && rleaf) {
        if (c.use_tokens) t = t + WR;
        cd = BASE;
        bevals += NQ * (int64_t)rt.count[R];
      } else {
        cd = SPLIT;
      }
    }
    if (cd == SPLIT) {
      nchild += rleaf ? 1 : 2;
    } else {
      Lp = Lp + WR * km;
      if (cd != FD) sc.v[2 + (cd - DH)] += 1;
    }
    counts[cd] += 1;
    code_out[off + j] = (int8_t)cd;
    p_out[off + j] = (int8_t)p;
  }
  if (any_fd) Gest[(int64_t)h * nQ + Q] = gest;
  cur.T[s] = t;
  cur.Lp[s] = Lp;
  if (nchild > 0) {
    sc.v[1] = qleaf ? 1 : 2;
    sc.v[0] = nchild * sc.v[1];
  }
  for (int k = 0; k < 4; ++k) sc.v[6 + k] = sc.v[2 + k] > 0 ? 1 : 0;
  cnt[s] = sc;
  for (int k = 0; k < 6; ++k)
    if (counts[k]) atomicAdd(&hcount[h * 6 + k], (unsigned long long)counts[k]);
  if (bevals) atomicAdd(base_evals, (unsigned long long)bevals);
}

struct SegCountPlus {
  __device__ __host__ SegCount operator()(const SegCount& a, const SegCount& b) const {
    SegCount r;
    for (int k = 0; k < 10; ++k) r.v[k] = a.v[k] + b.v[k];
    return r;
  }
};

__global__ void emit_kernel(int S, FrontierLevel cur, FrontierLevel nxt,
                            const int32_t* __restrict__ qleft, const int32_t* __restrict__ rleft,
                            const int8_t* __restrict__ code, const int8_t* __restrict__ porder,
                            const SegCount* __restrict__ cnt, const SegCount* __restrict__ incl,
                            WorkLists wl, LevelOffsets base) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const SegCount own = cnt[s];
  const SegCount in = incl[s];
  int ex[10];
  for (int k = 0; k < 10; ++k) ex[k] = in.v[k] - own.v[k];
  const int h = cur.h[s];
  const int Q = cur.Q[s];
  const int off = cur.off[s];
  const int len = cur.len[s];
  const bool qleaf = qleft[Q] < 0;
  const int nsegs = own.v[1];
  const int nch = nsegs ? own.v[0] / nsegs : 0;
  const int pb = ex[0];
  if (nsegs) {
    const int sb = ex[1];
    const double T = cur.T[s], Lp = cur.Lp[s];
    for (int k = 0; k < nsegs; ++k) {
      nxt.h[sb + k] = h;
      nxt.Q[sb + k] = qleaf ? Q : qleft[Q] + k;
      nxt.off[sb + k] = pb + k * nch;
      nxt.len[sb + k] = nch;
      nxt.T[sb + k] = T;
      nxt.Lp[sb + k] = Lp;
    }
  }
  int eb[4];
  for (int x = 0; x < 4; ++x) {
    eb[x] = base.ent[x] + ex[2 + x];
    if (own.v[2 + x] > 0) wl.grp[x][base.grp[x] + ex[6 + x]] = make_int4(h, Q, eb[x], own.v[2 + x]);
  }
  int kc = 0;
  for (int j = 0; j < len; ++j) {
    const int cd = code[off + j];
    const int R = cur.R[off + j];
    if (cd == SPLIT) {
      const int rl = rleft[R];
      const int nk = rl < 0 ? 1 : 2;
      for (int u = 0; u < nk; ++u) {
        const int kid = rl < 0 ? R : rl + u;
        for (int k = 0; k < nsegs; ++k) nxt.R[pb + k * nch + kc] = kid;
        ++kc;
      }
    } else if (cd != FD) {
      const int x = cd - DH;
      wl.ent[x][eb[x]++] = (R << 4) | porder[off + j];
    }
  }
}

}  // namespace

hipError_t launch_decide(int S, const FrontierLevel& cur, const TreeView& qt, const TreeView& rt,
                         const double* inv2h2, const double* inv4h2, const double* invh, int nQ,
                         const DecideConst& c, double* scratch_kmax, double* scratch_dmin2,
                         int8_t* code, int8_t* porder, double* Gest, SegCount* cnt,
                         unsigned long long* hcount, unsigned long long* base_evals,
                         float* policy_feat, hipStream_t s) {
  (void)policy_feat;
  hipLaunchKernelGGL(decide_kernel, dim3((unsigned)ceil_div(S, 64)), dim3(64), 0, s, S, cur, qt, rt,
                     inv2h2, inv4h2, invh, nQ, c, scratch_kmax, scratch_dmin2, code, porder, Gest,
                     cnt, hcount, base_evals);
  return hipGetLastError();
}

size_t scan_counts_temp_bytes(int S) {
  size_t bytes = 0;
  SegCount zero;
  for (int k = 0; k < 10; ++k) zero.v[k] = 0;
  (void)rocprim::inclusive_scan((void*)nullptr, bytes, (const SegCount*)nullptr, (SegCount*)nullptr,
                          (size_t)S, SegCountPlus());
  (void)zero;
  return bytes;
}

hipError_t scan_counts(int S, const SegCount* cnt, SegCount* incl, void* temp, size_t temp_bytes,
                       hipStream_t s) {
  size_t bytes = temp_bytes;
  return rocprim::inclusive_scan(temp, bytes, cnt, incl, (size_t)S, SegCountPlus(), s);
}

hipError_t launch_emit(int S, const FrontierLevel& cur, const FrontierLevel& nxt,
                       const int32_t* qleft, const int32_t* rleft, const int8_t* code,
                       const int8_t* porder, const SegCount* cnt, const SegCount* incl,
                       const WorkLists& wl, LevelOffsets base, hipStream_t s) {
  hipLaunchKernelGGL(emit_kernel, dim3((unsigned)ceil_div(S, 64)), dim3(64), 0, s, S, cur, nxt,
                     qleft, rleft, code, porder, cnt, incl, wl, base);
  return hipGetLastError();
}

}  // namespace gs
