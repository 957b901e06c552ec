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

// One-dimensional parts of the O(p^D) bounds for a scaled radius rho:
// a = sum_{n<p} rho^n / sqrt(n!) (left to right) and pw = rho^p, extended one
// order at a time.
struct TensorPart {
  double rho, a = 0.0, pw = 1.0;
  __device__ explicit TensorPart(double r) : rho(r) {}
  __device__ __forceinline__ void extend(const DecideConst& c, int p) {
    a = a + pw * c.isf[p - 1];
    pw = pw * rho;
  }
  // b = (rho^p / sqrt(p!)) / (1 - rho / sqrt(p+1)), inf when the ratio
  // rho / sqrt(p+1) reaches 1
  __device__ __forceinline__ double b(const DecideConst& c, int p) const {
    const double q = rho * c.isq[p];
    return q < 1.0 ? (pw * c.isf[p]) / (1.0 - q) : INFINITY;
  }
};

// sum_{k<D} x^k, left to right.
__device__ __forceinline__ double geometric(double x, int D) {
  double v = 0.0, pw = 1.0;
  for (int k = 0; k < D; ++k) {
    v = v + pw;
    pw = pw * x;
  }
  return v;
}

// O(p^D) far-field or local bound: W_R g (K b) sum_{k<D} (K a)^k, the
// product form of the tensor truncation with Cramer's inequality per factor.
__device__ __forceinline__ double tensor_bound(const DecideConst& c, double base_e, const TensorPart& t,
                                               int p) {
  const double b = t.b(c, p);
  if (b == INFINITY) return INFINITY;
  return base_e * ((c.kc * b) * geometric(c.kc * t.a, c.D));
}

// O(p^D) H2L bound: the dropped part of the double series over (m, n) with
// m or n >= p, rho = sqrt2 r on both sides.
__device__ __forceinline__ double tensor_h2l_bound(const DecideConst& c, double base_e, const TensorPart& tR,
                                                   const TensorPart& tQ, int p) {
  const double bR = tR.b(c, p), bQ = tQ.b(c, p);
  if (bR == INFINITY || bQ == INFINITY) return INFINITY;
  const double tail = bR * (tQ.a + bQ) + tR.a * bQ;
  return base_e * ((c.kc * tail) * geometric(c.kc * (tR.a * tQ.a), c.D));
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

__device__ __forceinline__ double need_fn(double E, double WR, double L, double W, double eps) {
  if (E == 0.0) return -WR;
  if (L == 0.0) return INFINITY;
  return (W * E) / (eps * L) - WR;
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

// Broadcast of lane j's value to the whole wave (v_readlane: register to
// register, no memory round trip).  j must be wave-uniform.
__device__ __forceinline__ int rl(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
__device__ __forceinline__ long long rl(long long v, int j) {
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), j);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), j);
  return ((long long)(unsigned)lo) | ((long long)hi << 32);
}
__device__ __forceinline__ double rl(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Smallest double a with fl(a / W) >= m (W > 0): correctly rounded division is
// monotone, so fl(a / W) >= m exactly when a >= astar.  m = +INFINITY (or NaN)
// gives +INFINITY.  -INFINITY, which sends the caller to the division itself,
// for m below the smallest normal double (there the quotient's rounding to
// zero or to a subnormal makes the threshold depend on W's last bits) and when
// the search does not settle within a few units in the last place.
__device__ double division_threshold(double m, double W) {
  if (!(m < INFINITY)) return INFINITY;
  if (!(m >= 2.2250738585072014e-308)) return -INFINITY;
  double a = m * W;
  if (a / W >= m) {
    for (int it = 0; it < 4; ++it) {
      const double b = nextafter(a, -INFINITY);
      if (b / W >= m)
        a = b;
      else
        return a;
    }
  } else {
    for (int it = 0; it < 4; ++it) {
      a = nextafter(a, INFINITY);
      if (a / W >= m) return a;
    }
  }
  return -INFINITY;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per pair of the level, all pairs at once: the token-independent values of
// the pair that involve its nodes' boxes, in the same arithmetic as the walk
// would form them.  prep is [5][npair]: W_R K(dmax), K(dmin), K(dmax),
// exp(-dmin^2 / 4h^2) (the bounds' Gaussian factor), W_R.
// Squared-distance bounds of the node pair (Q, R): the box bounds, or with
// node_bounds the tighter of those and the bounding-ball bounds.
__device__ __forceinline__ void pair_bounds(int Q, int R, const TreeView& qt, const TreeView& rt, int D,
                                            int node_bounds, double* dmin2_out, double* dmax2_out) {
  double dmin2, dmax2;
  box_dist2(qt.lo + (int64_t)Q * D, qt.hi + (int64_t)Q * D, rt.lo + (int64_t)R * D,
            rt.hi + (int64_t)R * D, D, &dmin2, &dmax2);
  if (node_bounds) {
    // the bounding balls about the box centres: every point pair is between
    // dc - rad_Q - rad_R and dc + rad_Q + rad_R apart; keep the tighter bounds
    const double* cQ = qt.ctr + (int64_t)Q * D;
    const double* cR = rt.ctr + (int64_t)R * D;
    double d2 = 0.0;
    for (int d = 0; d < D; ++d) {
      const double diff = cQ[d] - cR[d];
      d2 = d2 + diff * diff;
    }
    const double dc = sqrt(d2);
    const double rq = qt.rad[Q], rr = rt.rad[R];
    const double gap = (dc - rq) - rr;
    if (gap > 0.0) {
      const double g2 = gap * gap;
      if (g2 > dmin2) dmin2 = g2;
    }
    const double far = (dc + rq) + rr;
    const double f2 = far * far;
    if (f2 < dmax2) dmax2 = f2;
  }
  *dmin2_out = dmin2;
  *dmax2_out = dmax2;
}

__global__ __launch_bounds__(256) void pair_prep_kernel(int npair, FrontierLevel cur, TreeView qt,
                                                        TreeView rt, const double* __restrict__ inv2h2,
                                                        const double* __restrict__ inv4h2, int D,
                                                        int node_bounds, double* __restrict__ prep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npair) return;
  const int sg = cur.seg[i];
  const int h = cur.h[sg];
  const int Q = cur.Q[sg];
  const int R = cur.R[i];
  double dmin2, dmax2;
  pair_bounds(Q, R, qt, rt, D, node_bounds, &dmin2, &dmax2);
  const double i2 = inv2h2[h];
  const double kmax = own_exp(-dmax2 * i2);
  const double kmin = own_exp(-dmin2 * i2);
  const double g = own_exp(-dmin2 * inv4h2[h]);
  const double WR = rt.W[R];
  prep[i] = WR * kmax;
  prep[(int64_t)npair + i] = kmin;
  prep[2 * (int64_t)npair + i] = kmax;
  prep[3 * (int64_t)npair + i] = g;
  prep[4 * (int64_t)npair + i] = WR;
}

// One wave per segment, 64 pairs at a time, one pair per lane.
//
// Every quantity of a pair that does not depend on the token is computed by
// its lane, in parallel, and stays in that lane's registers: K(dmax), the
// finite-difference value and its token need, the bounds E_DH, E_DL, E_H2L of
// every order as prefix minima PM_X[p] = min(E_X(1..p)) (the first order whose
// bound meets maxerr is the first p with PM_X[p] <= maxerr, and there
// E_X(p) = PM_X[p]), and mstar, the smallest maxerr at which some series
// method beats DIRECT: the cost model of Figure 6 grows with the order, so
// method X can win only at an order p with c_X(p) <= c_Direct, and it reaches
// one exactly when PM_X[pmax_X] <= maxerr.  Below mstar the choice is DIRECT
// whatever the token, and "maxerr >= mstar" is tested without a division as
// "(eps (W_R + t)) L >= astar" (see division_threshold).
//
// The token rule (Figures 6-7) then walks the pairs in order with the whole
// wave in lockstep, reading pair j's values from lane j by register broadcast.
// A pair takes one of two paths.  The short one covers the finite-difference
// prune and every pair whose maxerr stays below the threshold at which a
// series method can be chosen (DIRECT: base case or split): a comparison with
// the token, maxerr's numerator, one comparison with the precomputed
// threshold and the token update, with the pair's code kept as a bit of a
// wave-uniform mask.  The long one, taken only above the threshold, runs the
// order search of bestMethod on lane j itself.  Gest_Q and Lpush_Q are summed
// in pair order inside the same walk (adding +0.0 for a pair that does not
// contribute, exact for these non-negative sums); counters come from the
// masks.  Every expression and its operation order is that of the
// single-threaded formulation, so the decisions and sums are identical to it.
// GEN: the learned policy or logging may be on; without them the walk
// compiles to the rule alone.  TEN: the O(p^D) bounds (tensor index sets)
// instead of the O(D^p) ones.
template <int P, bool GEN, bool TEN>
__global__ __launch_bounds__(64) void decide_kernel(int S, int n_first, FrontierLevel cur, TreeView qt,
                                                    TreeView rt, const double* __restrict__ inv2h2,
                                                    const double* __restrict__ inv4h2,
                                                    const double* __restrict__ invh, int nQ,
                                                    DecideConst c, int8_t* __restrict__ code_out,
                                                    int8_t* __restrict__ p_out,
                                                    double* __restrict__ Gest,
                                                    SegCount* __restrict__ cnt,
                                                    const float4* __restrict__ scores,
                                                    int16_t* __restrict__ feas_out,
                                                    const double* __restrict__ prep, int npair) {
  constexpr double kSqrt2 = 1.4142135623730951;
  // The long segments first (listed in cur.first), then the others.
  const int b = blockIdx.x;
  int s;
  if (b < n_first) {
    s = cur.first[b];
  } else {
    s = b - n_first;
    if (s >= S || (n_first > 0 && cur.len[s] >= kLongSegment)) return;
  }
  const int lane = threadIdx.x;
  const int h = cur.h[s];
  const int Q = cur.Q[s];
  const int off = cur.off[s];
  const int len = cur.len[s];
  if (len >= 2 * kLongSegment)
    __builtin_amdgcn_s_setprio(2);
  else if (len >= kLongSegment)
    __builtin_amdgcn_s_setprio(1);
  const double ih = invh[h];
  const bool qleaf = qt.left[Q] < 0;
  const double Wtot = rt.W[0];  // total reference weight (the root's)
  const int64_t NQ = qt.count[Q];
  const double rQ = qt.rinf[Q] * ih;
  __shared__ double4 sh_pair[64];  // need(E_FD), W_R, series threshold, FD value
  __shared__ double sh_lterm[64];  // W_R K(dmax)
  double* gest_at = Gest + (int64_t)h * nQ + Q;
  const double gest_in = *gest_at;

  // Lower bound L over Q, summed in pair order (each chunk's terms read one
  // chunk ahead).
  const double* p_lterm = prep;
  const double* p_kmin = prep + npair;
  const double* p_kmax = prep + 2 * (int64_t)npair;
  const double* p_g = prep + 3 * (int64_t)npair;
  const double* p_WR = prep + 4 * (int64_t)npair;
  double L = cur.Lp[s];
  {
    double nx = lane < len ? p_lterm[off + lane] : 0.0;
    for (int b0 = 0; b0 < len; b0 += 64) {
      const int n = len - b0 < 64 ? len - b0 : 64;
      const double lterm = nx;
      if (b0 + 64 < len) nx = b0 + 64 + lane < len ? p_lterm[off + b0 + 64 + lane] : 0.0;
      for (int j = 0; j < n; ++j) L = L + rl(lterm, j);
    }
  }
  if (c.mono && qt.wmin[Q] > L) L = qt.wmin[Q];

  double t = cur.T[s];
  double tdep = 0.0, twd = 0.0;  // this segment's token deposits and withdrawals
  double Lp = cur.Lp[s];
  double gest = gest_in;
  bool any_fd = false;
  int nFD = 0, nDH = 0, nDL = 0, nH2L = 0, nBASE = 0, nSPLIT = 0, nchild = 0;
  int ncalls = 0, nfall = 0;
  long long bevals = 0, dlchunks = 0;
  // When logging, every pair that reaches bestMethod needs its admitted
  // orders: no DIRECT shortcut.
  const bool all_orders = GEN && c.log_feas != 0;
  const bool learned = GEN && c.use_fmm && c.policy;
  // Cost tables of the segment, lane k holding order k: c_DH(k) = N_Q D^(k+1),
  // c_H2L(k) = D^(2k+1) (Figure 6).
  const long long c0_lane = lane >= 1 && lane <= P ? sat_mul(NQ, c.cterm[lane]) : kInfCost;
  const long long c2_lane = lane >= 1 && lane <= P ? c.ch2l[lane] : kInfCost;
  __shared__ double sh_pm[64][3 * P];      // PM_DH, PM_DL, PM_H2L of each pair
  for (int b0 = 0; b0 < len; b0 += 64) {
    const int n = len - b0 < 64 ? len - b0 : 64;
    double lterm = 0.0, fdval = 0.0, nd = 0.0, WR = 0.0, astar = INFINITY, thr = INFINITY;
    int NR = 0, rleaf = 0, Rid = 0;
    long long c3 = 0;
    int kstar = 0;  // learned policy: cheapest predicted action (3 = recurse)
    float4 psc = make_float4(0.f, 0.f, 0.f, 0.f);  // its predicted costs
    double pm0[P], pm1[P], pm2[P];
#pragma unroll
    for (int p = 0; p < P; ++p) pm0[p] = pm1[p] = pm2[p] = INFINITY;
    if (lane < n) {
      const int64_t pi = off + b0 + lane;
      const int R = cur.R[pi];
      WR = p_WR[pi];
      const double kmax = p_kmax[pi];
      const double kmin = p_kmin[pi];
      NR = rt.count[R];
      Rid = R;
      if (GEN && scores) {
        // ties go to the earlier of DH, DL, H2L, recurse
        const float4 sc = scores[off + b0 + lane];
        psc = sc;
        float sb = sc.x;
        if (sc.y < sb) { kstar = 1; sb = sc.y; }
        if (sc.z < sb) { kstar = 2; sb = sc.z; }
        if (sc.w < sb) { kstar = 3; sb = sc.w; }
      }
      rleaf = rt.left[R] < 0 ? 1 : 0;
      lterm = p_lterm[pi];
      fdval = 0.5 * (WR * (kmin + kmax));
      nd = need_fn(0.5 * (WR * (kmin - kmax)), WR, L, Wtot, c.eps_alg);
      if (c.use_fmm) {
        const double g = p_g[pi];
        const double rR = rt.rinf[R] * ih;
        const double base_e = WR * g;
        double m0 = INFINITY, m1 = INFINITY, m2 = INFINITY;
        if constexpr (TEN) {
          // O(p^D) bounds: a = sum_{n<p} rho^n / sqrt(n!) grows by one term
          // per order; b = rho^p / sqrt(p!) / (1 - rho / sqrt(p+1)).
          TensorPart tR(rR), tQ(rQ), tR2(kSqrt2 * rR), tQ2(kSqrt2 * rQ);
#pragma unroll
          for (int p = 1; p <= P; ++p) {
            tR.extend(c, p);
            tQ.extend(c, p);
            tR2.extend(c, p);
            tQ2.extend(c, p);
            const double e0 = (c.fmm_mask & 1) ? tensor_bound(c, base_e, tR, p) : INFINITY;
            const double e1 = (c.fmm_mask & 2) ? tensor_bound(c, base_e, tQ, p) : INFINITY;
            const double e2 = (c.fmm_mask & 4) ? tensor_h2l_bound(c, base_e, tR2, tQ2, p) : INFINITY;
            m0 = e0 < m0 ? e0 : m0;
            m1 = e1 < m1 ? e1 : m1;
            m2 = e2 < m2 ? e2 : m2;
            pm0[p - 1] = m0;
            pm1[p - 1] = m1;
            pm2[p - 1] = m2;
          }
        } else {
#pragma unroll
          for (int p = 1; p <= P; ++p) {
            const double bc = base_e * c.bconst[p];
            const double e0 = (c.fmm_mask & 1) ? bc * powi(rR, p) : INFINITY;
            const double e1 = (c.fmm_mask & 2) ? bc * powi(rQ, p) : INFINITY;
            double e2 = INFINITY;
            if (c.fmm_mask & 4) {
              const double sq = kSqrt2 * rQ;
              const double itail = sq <= 1.0 ? 1.0 : powi(sq, p - 1);
              const double second = (powi(kSqrt2 * rR, p) * c.binomD[p]) * itail;
              e2 = bc * (powi(rQ, p) + second);
            }
            m0 = e0 < m0 ? e0 : m0;
            m1 = e1 < m1 ? e1 : m1;
            m2 = e2 < m2 ? e2 : m2;
            pm0[p - 1] = m0;
            pm1[p - 1] = m1;
            pm2[p - 1] = m2;
          }
        }
        const int64_t cdir = sat_mul(c.D, sat_mul(NQ, (int64_t)NR));
        c3 = cdir;
        double mstar = INFINITY;
#pragma unroll
        for (int p = 1; p <= P; ++p) {
          const int64_t c1p = sat_mul((int64_t)NR, c.cterm[p]);
          if (sat_mul(NQ, c.cterm[p]) <= cdir) mstar = pm0[p - 1] < mstar ? pm0[p - 1] : mstar;
          if (c1p <= cdir) mstar = pm1[p - 1] < mstar ? pm1[p - 1] : mstar;
          if (c.ch2l[p] <= cdir) mstar = pm2[p - 1] < mstar ? pm2[p - 1] : mstar;
        }
        astar = all_orders ? -INFINITY : division_threshold(mstar, Wtot);
        thr = astar;
        if (learned) {
          // some series method is admitted at some order exactly when
          // maxerr reaches the smallest of the bounds; a preferred recursion
          // needs no order search
          if (kstar == 3) {
            thr = INFINITY;
          } else {
            double mk = pm0[P - 1] < pm1[P - 1] ? pm0[P - 1] : pm1[P - 1];
            mk = pm2[P - 1] < mk ? pm2[P - 1] : mk;
            thr = division_threshold(mk, Wtot);
          }
        }
      }
    }
    const unsigned long long base_ok = qleaf ? __ballot(lane < n && rleaf) : 0ull;
    const unsigned long long kfall = learned ? __ballot(lane < n && kstar != 3) : 0ull;
    // Pair values the walk reads, staged in LDS and read back as broadcasts;
    // the bounds as one row per pair, read across the lanes.
    __syncthreads();
    if (lane < n) {
      sh_pair[lane] = make_double4(nd, WR, thr, fdval);
      sh_lterm[lane] = lterm;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        sh_pm[lane][p] = pm0[p];
        sh_pm[lane][P + p] = pm1[p];
        sh_pm[lane][2 * P + p] = pm2[p];
      }
    }
    __syncthreads();
    // The token rule, pair by pair, the wave in lockstep.
    unsigned long long m_fd = 0, m_slow = 0, m_base = 0;
    int my_code = -1, my_p = 0, my_feas = 0;
    int j = 0;
    while (j < n) {
      // Short path until a pair reaches the series threshold.
      double a = 0.0, WRj = 0.0, ltj = 0.0;
      bool slow = false;
      double4 nx = sh_pair[j];  // read one pair ahead
      double nx_lt = sh_lterm[j];
      for (; j < n; ++j) {
        const double4 pv = nx;
        ltj = nx_lt;
        nx = sh_pair[(j + 1) & 63];
        nx_lt = sh_lterm[(j + 1) & 63];
        WRj = pv.y;
        const double tt = c.use_tokens ? t : 0.0;
        a = (c.eps_alg * (WRj + tt)) * L;
        const bool fd = pv.x <= tt;
        if (!fd && a >= pv.z) {
          slow = true;
          break;
        }
        // finite difference, or DIRECT below the series threshold (and the
        // learned policy's recursion): base case if both nodes are leaves,
        // else split
        const unsigned long long bit = 1ull << j;
        const bool base = !fd && (base_ok & bit);
        if (c.use_tokens) {
          t = fd ? t - pv.x : (base ? t + WRj : t);
          const double dv = fd ? -pv.x : (base ? WRj : 0.0);  // the token change
          tdep = tdep + (dv > 0.0 ? dv : 0.0);
          twd = twd + (dv < 0.0 ? -dv : 0.0);
        }
        m_fd |= fd ? bit : 0ull;
        m_base |= base ? bit : 0ull;
        gest = gest + (fd ? pv.w : 0.0);
        Lp = Lp + (!fd && !base ? 0.0 : ltj);
        any_fd = any_fd || fd;
      }
      if (!slow) break;
      // bestMethod (Figure 6) at maxerr for pair j: its bounds across the
      // lanes, the admitted order of each method counted from one ballot.
      m_slow |= 1ull << j;
      const double maxerr = a / Wtot;
      const double pmv = lane < 3 * P ? sh_pm[j][lane] : INFINITY;
      // token need of every bound (independent of the token: computed beside
      // maxerr, read back for the chosen one)
      const double needv = need_fn(pmv, WRj, L, Wtot, c.eps_alg);
      const unsigned long long gt = __ballot(lane < 3 * P && pmv > maxerr);
      const unsigned long long fm = (1ull << P) - 1;
      const int n0 = __popcll(gt & fm), n1 = __popcll((gt >> P) & fm),
                n2 = __popcll((gt >> (2 * P)) & fm);
      int q0 = n0 < P ? n0 + 1 : 0, q1 = n1 < P ? n1 + 1 : 0, q2 = n2 < P ? n2 + 1 : 0;
      int cd = -1, p = 0, xs = 0;
      bool rule = c.use_fmm != 0;
      if (learned) {
        // The learned policy: the cheapest predicted of the admitted actions
        // (each series method whose bound admits an order, at its smallest
        // such order, and recursion, always admitted); ties go to the earlier
        // of DH, DL, H2L, recurse.  An override is counted when the overall
        // cheapest prediction was not admitted.
        rule = false;
        const int kj = rl(kstar, j);
        if (kj != 3) {
          const float sk[4] = {__int_as_float(rl(__float_as_int(psc.x), j)),
                               __int_as_float(rl(__float_as_int(psc.y), j)),
                               __int_as_float(rl(__float_as_int(psc.z), j)),
                               __int_as_float(rl(__float_as_int(psc.w), j))};
          const int qv[3] = {q0, q1, q2};
          int best = 3;
          float sb = sk[3];
          for (int k = 2; k >= 0; --k)
            if (qv[k] && sk[k] <= sb) {
              best = k;
              sb = sk[k];
            }
          if (best != kj) ++nfall;
          if (best < 3) {
            cd = DH + best;
            p = qv[best];
            xs = best;
          }
        }
      }
      // (without the policy, thr is astar and a >= astar holds here)
      if (rule && (!GEN || all_orders || a >= rl(astar, j))) {
        // c_DL(q1) = N_R c_term(q1) of pair j (its N_R read from lane j)
        const int64_t c0 = q0 ? rl(c0_lane, q0) : kInfCost;
        const int64_t c1 = q1 ? sat_mul((int64_t)__builtin_amdgcn_readlane(NR, j), c.cterm[q1]) : kInfCost;
        const int64_t c2 = q2 ? rl(c2_lane, q2) : kInfCost;
        const int64_t cd3 = rl(c3, j);
        int64_t best = c0 < c1 ? c0 : c1;
        best = c2 < best ? c2 : best;
        best = cd3 < best ? cd3 : best;
        if (q0 && c0 == best) {
          cd = DH;
          p = q0;
          xs = 0;
        } else if (q1 && c1 == best) {
          cd = DL;
          p = q1;
          xs = 1;
        } else if (q2 && c2 == best) {
          cd = H2L;
          p = q2;
          xs = 2;
        }
        if (GEN && c.log_feas && c.explore > 0.0) {
          // Exploration while logging: for a fixed pseudo-random share of
          // the pairs, an admitted action drawn uniformly (each admitted
          // series method at its order, or the direct path) replaces the
          // rule's, so that the log also holds costs the rule never incurs.
          unsigned long long x = ((unsigned long long)h << 56) ^ ((unsigned long long)Q << 28) ^
                                 (unsigned long long)rl(Rid, j);
          x += 0x9e3779b97f4a7c15ull;
          x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
          x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
          x ^= x >> 31;
          if ((double)(x >> 11) * 0x1.0p-53 < c.explore) {
            const int ncand = (q0 ? 1 : 0) + (q1 ? 1 : 0) + (q2 ? 1 : 0) + 1;
            int pick = (int)((x & 0x3ff) * (unsigned long long)ncand >> 10);
            cd = -1;
            p = 0;
            if (q0 && pick-- == 0) {
              cd = DH;
              p = q0;
              xs = 0;
            } else if (q1 && pick-- == 0) {
              cd = DL;
              p = q1;
              xs = 1;
            } else if (q2 && pick-- == 0) {
              cd = H2L;
              p = q2;
              xs = 2;
            }
          }
        }
        if (GEN && c.log_feas && lane == j) my_feas = 0x8000 | q0 | (q1 << 4) | (q2 << 8);
      }
      if (cd >= 0) {
        if (c.use_tokens) {
          const double v = rl(needv, xs * P + p - 1);
          t = t - v;
          tdep = tdep + (v < 0.0 ? -v : 0.0);
          twd = twd + (v > 0.0 ? v : 0.0);
        }
      } else if (base_ok & (1ull << j)) {
        if (c.use_tokens) {
          t = t + WRj;
          tdep = tdep + WRj;
        }
        cd = BASE;
      } else {
        cd = SPLIT;
      }
      nDH += cd == DH;
      nDL += cd == DL;
      nH2L += cd == H2L;
      nBASE += cd == BASE;
      nSPLIT += cd == SPLIT;
      if (lane == j) {
        my_code = cd;
        my_p = p;
      }
      Lp = Lp + (cd == SPLIT ? 0.0 : ltj);
      ++j;
    }
    const unsigned long long bitl = 1ull << lane;
    int code;
    if (m_fd & bitl) code = FD;
    else if (m_slow & bitl) code = my_code;
    else if (m_base & bitl) code = BASE;
    else code = SPLIT;
    const unsigned long long live = n == 64 ? ~0ull : (1ull << n) - 1;
    const unsigned long long m_fast = live & ~(m_fd | m_slow);
    nFD += __popcll(m_fd);
    nBASE += __popcll(m_base);
    nSPLIT += __popcll(m_fast & ~m_base);
    if (learned) {
      ncalls += __popcll(live & ~m_fd);
      nfall += __popcll(m_fast & kfall);
    }
    const bool act = lane < n;
    const unsigned long long m_split = __ballot(act && code == SPLIT);
    const unsigned long long m_rleaf = __ballot(act && rleaf);
    nchild += __popcll(m_split & m_rleaf) + 2 * __popcll(m_split & ~m_rleaf);
    if (__ballot(act && code == BASE))
      bevals += wave_sum_ll(act && code == BASE ? (long long)NQ * NR : 0ll);
    if (__ballot(act && code == DL)) dlchunks += wave_sum_ll(act && code == DL ? (NR + 63) / 64 : 0);
    if (act) {
      code_out[off + b0 + lane] = (int8_t)code;
      p_out[off + b0 + lane] = (int8_t)((m_slow & bitl) ? my_p : 0);
      if (GEN && feas_out) feas_out[off + b0 + lane] = (int16_t)((m_slow & bitl) ? my_feas : 0);
    }
  }
  if (lane != 0) return;
  if (any_fd) *gest_at = gest;
  if (c.tok) {
    if (tdep != 0.0) atomicAdd(c.tok, tdep);
    if (twd != 0.0) atomicAdd(c.tok + 1, twd);
  }
  cur.T[s] = t;
  cur.Lp[s] = Lp;
  SegCount sc;
  sc.v[1] = nchild > 0 ? (qleaf ? 1 : 2) : 0;
  sc.v[0] = nchild * sc.v[1];
  sc.v[2] = nDH;
  sc.v[3] = nDL;
  sc.v[4] = nH2L;
  sc.v[5] = nBASE;
  sc.v[6] = nDH > 0;
  sc.v[7] = nDL > 0;
  sc.v[8] = nH2L > 0;
  sc.v[9] = nBASE > 0;
  sc.v[10] = nFD;
  sc.v[11] = nSPLIT;
  sc.v[12] = bevals;
  sc.v[13] = ncalls;
  sc.v[14] = nfall;
  sc.v[15] = (nDH + kDHSliceEntries - 1) / kDHSliceEntries;
  sc.v[16] = (dlchunks + kDLSliceChunks - 1) / kDLSliceChunks;
  sc.v[17] = nchild >= kLongSegment ? sc.v[1] : 0;
  cnt[s] = sc;
}

struct SegCountPlus {
  __device__ __host__ SegCount operator()(const SegCount& a, const SegCount& b) const {
    SegCount r;
    for (int k = 0; k < 18; ++k) r.v[k] = a.v[k] + b.v[k];
    return r;
  }
};

// Exclusive prefix sum over the 64 lanes of a wave; *total receives the sum.
__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
  const int lane = threadIdx.x & 63;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

// One wave per segment: next-level segments and pairs (children in the same
// left-to-right order) and typed work entries, positions by wave prefix sums.
__global__ __launch_bounds__(64) void emit_kernel(int S, FrontierLevel cur, FrontierLevel nxt,
                                                  const int32_t* __restrict__ qleft,
                                                  const int32_t* __restrict__ rleft,
                                                  const int8_t* __restrict__ code,
                                                  const int8_t* __restrict__ porder,
                                                  const SegCount* __restrict__ cnt,
                                                  const SegCount* __restrict__ incl,
                                                  const int32_t* __restrict__ rcount, WorkLists wl,
                                                  LevelOffsets base,
                                                  unsigned long long* __restrict__ hcount,
                                                  unsigned long long* __restrict__ ev) {
  const int s = blockIdx.x;
  if (s >= S) return;
  const int lane = threadIdx.x;
  const SegCount own = cnt[s];
  const SegCount in = incl[s];
  // totals were checked on the host to fit 32-bit offsets
  int ex[10];
  for (int k = 0; k < 10; ++k) ex[k] = (int)(in.v[k] - own.v[k]);
  const int h = cur.h[s];
  const int Q = cur.Q[s];
  const int off = cur.off[s];
  const int len = cur.len[s];
  const bool qleaf = qleft[Q] < 0;
  if (lane == 0) {
    // Counters of the bandwidth run this segment ends (+ its inclusive sums)
    // or starts (- the sums before it): a run's net is its own total.
    const int sl[6] = {10, 2, 3, 4, 5, 11};  // FD, DH, DL, H2L, BASE, SPLIT
    unsigned long long* hc = hcount + h * 6;
    if (s == S - 1 || cur.h[s + 1] != h)
      for (int k = 0; k < 6; ++k)
        if (in.v[sl[k]]) atomicAdd(&hc[k], (unsigned long long)in.v[sl[k]]);
    if (s > 0 && cur.h[s - 1] != h) {
      const SegCount before = incl[s - 1];
      for (int k = 0; k < 6; ++k)
        if (before.v[sl[k]]) atomicAdd(&hc[k], 0ull - (unsigned long long)before.v[sl[k]]);
    }
    if (s == S - 1) {
      if (in.v[12]) atomicAdd(&ev[0], (unsigned long long)in.v[12]);
      if (in.v[13]) atomicAdd(&ev[2], (unsigned long long)in.v[13]);
      if (in.v[14]) atomicAdd(&ev[3], (unsigned long long)in.v[14]);
    }
  }
  const int nsegs = (int)own.v[1];
  const int nch = nsegs ? (int)(own.v[0] / nsegs) : 0;
  const int pb = ex[0];
  const int sb = ex[1];
  if (lane < nsegs && nch >= kLongSegment) nxt.first[(int)(in.v[17] - own.v[17]) + lane] = sb + lane;
  if (lane < nsegs) {
    nxt.h[sb + lane] = h;
    nxt.Q[sb + lane] = qleaf ? Q : qleft[Q] + lane;
    nxt.off[sb + lane] = pb + lane * nch;
    nxt.len[sb + lane] = nch;
    nxt.T[sb + lane] = cur.T[s];
    nxt.Lp[sb + lane] = cur.Lp[s];
  }
  int eb[4];
  for (int x = 0; x < 4; ++x) {
    eb[x] = base.ent[x] + ex[2 + x];
    if (lane == 0 && own.v[2 + x] > 0)
      wl.grp[x][base.grp[x] + ex[6 + x]] = make_int4(h, Q, eb[x], (int)own.v[2 + x]);
  }
  if (own.v[2] > 0) {
    // DH slices: runs of kDHSliceEntries entries
    const int g = base.grp[0] + ex[6];
    const int sb = base.slc[0] + (int)(in.v[15] - own.v[15]);
    const int ne = (int)own.v[2], ns = (int)own.v[15];
    for (int k = lane; k < ns; k += 64) {
      const int e0 = k * kDHSliceEntries;
      wl.dh_slice[sb + k] = make_int4(g, eb[0] + e0, min(kDHSliceEntries, ne - e0), k);
    }
    if (lane == 0) wl.dh_first[g] = sb;
  }
  int dl_run = 0;  // chunks of this segment's DL entries so far
  int kc = 0;
  for (int b0 = 0; b0 < len; b0 += 64) {
    const bool act = b0 + lane < len;
    const int cd = act ? code[off + b0 + lane] : -1;
    const int R = act ? cur.R[off + b0 + lane] : 0;
    const int rl = act ? rleft[R] : -1;
    const int nk = cd == SPLIT ? (rl < 0 ? 1 : 2) : 0;
    int tot;
    const int kp = wave_excl_scan(nk, &tot);
    for (int u = 0; u < nk; ++u) {
      const int kid = rl < 0 ? R : rl + u;
      for (int k = 0; k < nsegs; ++k) {
        const int o = pb + k * nch + kc + kp + u;
        nxt.R[o] = kid;
        nxt.seg[o] = sb + k;
      }
    }
    kc += tot;
    for (int x = 0; x < 4; ++x) {
      const int f = cd == DH + x ? 1 : 0;
      int tx;
      const int ep = wave_excl_scan(f, &tx);
      if (f) wl.ent[x][eb[x] + ep] = (R << 4) | porder[off + b0 + lane];
      if (x == 1 && tx) {
        const int ch = f ? (rcount[R] + 63) / 64 : 0;
        int tch;
        const int cp = wave_excl_scan(ch, &tch);
        if (f) wl.dl_cpre[eb[1] + ep] = dl_run + cp;
        dl_run += tch;
      }
      eb[x] += tx;
    }
  }
  if (own.v[3] > 0) {
    // DL slices: runs of kDLSliceChunks chunks over the entries in order
    const int g = base.grp[1] + ex[7];
    const int sb = base.slc[1] + (int)(in.v[16] - own.v[16]);
    const int ns = (int)own.v[16];
    for (int k = lane; k < ns; k += 64)
      wl.dl_slice[sb + k] = make_int4(g, k * kDLSliceChunks, min(dl_run, (k + 1) * kDLSliceChunks), 0);
    if (lane == 0) wl.dl_first[g] = make_int2(sb, ns);
  }
}

// The FP64 operations the decisions are made of, one element per thread:
// own_exp(x), x / y and sqrt(y), in the same compilation settings as the
// decide kernels (no contraction), so that a test can compare their bits with
// the host's correctly rounded results.
__global__ __launch_bounds__(256) void decision_arith_kernel(const double* __restrict__ x,
                                                             const double* __restrict__ y, int64_t n,
                                                             double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = own_exp(x[i]);
  out[n + i] = x[i] / y[i];
  out[2 * n + i] = sqrt(y[i]);
}

}  // namespace

hipError_t launch_decision_arith(const double* x, const double* y, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(decision_arith_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n, out);
  return hipGetLastError();
}

// Far-first order of each segment (a best-first walk of a query node's
// reference list): decreasing dmin^2, ties by increasing R.  Pair i's
// position is the number of pairs of its segment that precede it in that
// order (every R occurs once per segment, so positions are a permutation).
__global__ __launch_bounds__(256) void far_first_key_kernel(int npair, FrontierLevel cur, TreeView qt,
                                                            TreeView rt, int D, int node_bounds,
                                                            double* __restrict__ d2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npair) return;
  double dmin2, dmax2;
  pair_bounds(cur.Q[cur.seg[i]], cur.R[i], qt, rt, D, node_bounds, &dmin2, &dmax2);
  d2[i] = dmin2;
}

__global__ __launch_bounds__(256) void far_first_place_kernel(int npair, FrontierLevel cur,
                                                              const double* __restrict__ d2,
                                                              int32_t* __restrict__ r_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npair) return;
  const int sg = cur.seg[i];
  const int o = cur.off[sg], n = cur.len[sg];
  const double di = d2[i];
  const int Ri = cur.R[i];
  int rank = 0;
  for (int j = o; j < o + n; ++j) {
    const double dj = d2[j];
    const int Rj = cur.R[j];
    rank += (dj > di || (dj == di && Rj < Ri)) ? 1 : 0;
  }
  r_out[o + rank] = Ri;
}

hipError_t launch_far_first_order(int npair, const FrontierLevel& cur, const TreeView& qt, const TreeView& rt,
                                  int D, int node_bounds, double* d2, int32_t* r_tmp, hipStream_t s) {
  if (npair <= 0) return hipSuccess;
  const dim3 grid((unsigned)ceil_div(npair, 256));
  hipLaunchKernelGGL(far_first_key_kernel, grid, dim3(256), 0, s, npair, cur, qt, rt, D, node_bounds, d2);
  hipLaunchKernelGGL(far_first_place_kernel, grid, dim3(256), 0, s, npair, cur, d2, r_tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(cur.R, r_tmp, sizeof(int32_t) * npair, hipMemcpyDeviceToDevice, s);
}

hipError_t launch_decide(int S, int n_first, const FrontierLevel& cur, const TreeView& qt, const TreeView& rt,
                         const double* inv2h2, const double* inv4h2, const double* invh, int nQ,
                         const DecideConst& c, int8_t* code, int8_t* porder, double* Gest,
                         SegCount* cnt, const float4* scores, int16_t* feas, double* prep,
                         int npair, hipStream_t s) {
  hipLaunchKernelGGL(pair_prep_kernel, dim3((unsigned)ceil_div(npair, 256)), dim3(256), 0, s, npair,
                     cur, qt, rt, inv2h2, inv4h2, c.D, c.node_bounds, prep);
  const bool gen = c.policy != 0 || c.log_feas != 0 || scores != nullptr || feas != nullptr;
  // the policy and its logging serve the O(D^p) path only
  if (gen && c.tensor) return hipErrorInvalidValue;
#define GS_DECIDE(PP)                                                                                \
  case PP:                                                                                          \
    if (c.tensor)                                                                                   \
      hipLaunchKernelGGL((decide_kernel<PP, false, true>), dim3((unsigned)(S + n_first)), dim3(64), \
                         0, s, S, n_first, cur, qt, rt, inv2h2, inv4h2, invh, nQ, c, code, porder,  \
                         Gest, cnt, scores, feas, prep, npair);                                     \
    else if (gen)                                                                                   \
      hipLaunchKernelGGL((decide_kernel<PP, true, false>), dim3((unsigned)(S + n_first)), dim3(64), \
                         0, s, S, n_first, cur, qt, rt, inv2h2, inv4h2, invh, nQ, c, code, porder,  \
                         Gest, cnt, scores, feas, prep, npair);                                     \
    else                                                                                            \
      hipLaunchKernelGGL((decide_kernel<PP, false, false>), dim3((unsigned)(S + n_first)),          \
                         dim3(64), 0, s, S, n_first, cur, qt, rt, inv2h2, inv4h2, invh, nQ, c, code,\
                         porder, Gest, cnt, scores, feas, prep, npair);                             \
    break;
  switch (c.P) {
    GS_DECIDE(1) GS_DECIDE(2) GS_DECIDE(3) GS_DECIDE(4) GS_DECIDE(5)
    GS_DECIDE(6) GS_DECIDE(7) GS_DECIDE(8) GS_DECIDE(9) GS_DECIDE(10)
    default:
      return hipErrorInvalidValue;
  }
#undef GS_DECIDE
  return hipGetLastError();
}

size_t scan_counts_temp_bytes(int S) {
  size_t bytes = 0;
  SegCount zero;
  for (int k = 0; k < 18; ++k) zero.v[k] = 0;
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
                       const int32_t* rcount, const WorkLists& wl, LevelOffsets base,
                       unsigned long long* hcount, unsigned long long* ev, hipStream_t s) {
  hipLaunchKernelGGL(emit_kernel, dim3((unsigned)S), dim3(64), 0, s, S, cur, nxt, qleft, rleft,
                     code, porder, cnt, incl, rcount, wl, base, hcount, ev);
  return hipGetLastError();
}

}  // namespace gs
