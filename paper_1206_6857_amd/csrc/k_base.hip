// Exhaustive base cases of the dual-tree traversal (DITOBase, Figure 7),
// fused over bandwidths:
//     gx[h][q] = sum over base pairs (Q, R) of h, r in R:  w_r exp(-|x_q - x_r|^2 / 2h^2),
// for q in the leaf Q.
//
// The traversal records base pairs per (h, Q).  The same leaf pair is usually
// a base case for several neighbouring bandwidths, and |x_q - x_r|^2 does not
// depend on h, so the entries are regrouped by (Q, block of 16 bandwidths, R)
// with a 16-bit mask of the block's bandwidths that need the pair: a radix
// sort of (Q, block, R) keys, then an OR reduction by key.  (On mixtures of
// 10^6 points with 64 log-spaced bandwidths a leaf pair is a base case for
// 11 of a block's 16 bandwidths on average at D = 8, 8.7 at D = 5, against
// 6.9 and 5.9 of 8 with blocks of 8.)  A run is the set of
// regrouped entries of one (Q, block); runs are cut into slices of at most S
// entries, S chosen so that there are many more slices than SIMDs (the runs of
// dense clusters hold hundreds of entries, the others a few).
//
// One wave handles one slice: lanes hold the points of Q, the wave sweeps the
// reference leaves of its entries, and every point pair's squared distance
// feeds one exp2 per bandwidth of the entry's mask.  Reference records are read
// with wave-uniform addresses (scalar loads, several records per load, the
// next batch requested before the current one is used); each leaf's records
// are padded with zero-weight records to a multiple of 4.  A run of one slice
// writes gx directly; otherwise every slice writes its partial sums and a
// second kernel adds them in slice order.  Every gx[h][q] is written once and
// the result is deterministic.
//
// Precision: reference coordinates are stored relative to their leaf centre
// in float (u_r = x_r - c_R); each lane forms u_q = x_q - c_R in double before
// rounding to float, so u_q - u_r is accurate to ~2^-24 of the pair's extent.
// Every term of a leaf pair is scaled by exp(+d_box^2 / 2h^2), where d_box is
// the distance from x_q to R's bounding box (a lower bound of |x_q - x_r|, so
// each scaled term is <= 1 and far pairs stay out of the float underflow
// range); the leaf-pair sum is unscaled in double precision.  Weights are
// stored divided by the largest weight.  Where the box distance is a poor
// bound (a query inside a large, sparsely filled box, e.g. in 8 dimensions),
// every scaled term can still underflow: for a bandwidth whose scaled sum ends
// below 2^-60 on any lane, the wave sweeps the leaf again with each lane's
// shift taken from its smallest squared distance to the leaf's points (one
// distance-only sweep), so that the largest term is 1.
// Padding records sit far away (coordinates 1e18, weight 0): their terms are
// exactly 0 and they never give the smallest distance.
#include <cstring>  // rocprim uses memset without including it
#include <rocprim/rocprim.hpp>

#include <algorithm>

#include "gs_series.h"

namespace gs {

namespace {

constexpr int kW = 64;
constexpr int kHB = kBaseHB;  // bandwidths per block
constexpr int kPad = 4;  // records per leaf are padded to a multiple of this
constexpr int kResidentWaves = 4 * 4 * 256;  // base_fused_kernel: 4 waves per SIMD
constexpr int kBaseWaves = 4;                 // waves per workgroup of base_fused_kernel
constexpr int kReduceThreads = 256;           // base_reduce_kernel
constexpr uint64_t kAgeStep = 30000;          // 300 us of the 100 MHz real-time clock
constexpr int kEntryCost = 256;               // issue slots of an entry's set-up (box distance, mask)

constexpr float kFarPad = 1e18f;  // coordinate of the padding records

// MFMA distance records (file comment): groups of kMG references; a group
// holds, for k = 0, 2, 4, ..: 64 floats (a_k of its 32 references, then
// a_{k+1}), then the 32 weights.  a = (-2 u_r, 1, |u_r|^2, 0 padding).
constexpr int kMG = 32;
constexpr float kFarNorm = 1e30f;  // |u_r|^2 of a padding reference
__host__ __device__ constexpr int mfma_k2(int D) { return (D + 3) / 2 * 2; }
__host__ __device__ constexpr int mfma_group_floats(int D) { return kMG * mfma_k2(D) + kMG; }
// Dimensions whose compiled base tiles take distances from MFMA.
constexpr bool mfma_dim(int DT) { return DT >= 2; }
// Rounding bound of the expansion |u_q|^2 + |u_r|^2 - 2 u_q.u_r in float,
// in units of 2^-24 (|u_q| + |u_r|)^2: the two norms are summed exactly in
// double from the same float coordinates the products use and rounded once
// (one unit for both, |u_q|^2 + |u_r|^2 <= (|u_q| + |u_r|)^2; |u_q|^2 - T_q
// likewise, T_q being the float shift the unscaling uses); the K2 products
// and the K2 additions of the MFMA chain at most K2 + 1 units of their
// absolute sum, which is <= (|u_q| + |u_r|)^2; one more for the bound's own
// rounding.
template <int D>
constexpr int kMfmaErrC = mfma_k2(D) + 3;
// Largest relative error of a kernel term admitted from the expansion.
constexpr float kMfmaTau = 0x1p-12f;

// Every record of the array set to a padding record: far coordinates, weight 0.
__global__ void pad_records_kernel(float* __restrict__ rec, int64_t n_floats, int D, int rs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_floats) return;
  rec[i] = (int)(i % rs) < D ? kFarPad : 0.0f;
}

// Every MFMA record group set to padding references: a = (0, 1, 1e30, 0),
// weight 0, so that a padding reference's squared distance is ~1e30 and its
// term exactly 0.
__global__ void mfma_pad_kernel(float* __restrict__ mrec, int64_t n_floats, int D) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_floats) return;
  const int gf = mfma_group_floats(D), k2 = mfma_k2(D);
  const int pos = (int)(i % gf);
  float v = 0.0f;
  if (pos < kMG * k2) {
    const int k = 2 * (pos / 64) + (pos % 64) / kMG;
    v = k == D ? 1.0f : k == D + 1 ? kFarNorm : 0.0f;
  }
  mrec[i] = v;
}

// Groups per leaf (0 for internal nodes), and the leaves' largest |u_r|^2 cleared.
__global__ void mfma_groups_kernel(const int32_t* __restrict__ left, const int32_t* __restrict__ count,
                                   int n_nodes, int32_t* __restrict__ ngroups, float* __restrict__ rmax2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  ngroups[i] = left[i] < 0 ? (count[i] + kMG - 1) / kMG : 0;
  rmax2[i] = 0.0f;
}

// One thread per reference point: its augmented vector and weight in its
// leaf's groups, and the leaf's largest |u_r|^2 (the same float coordinates
// as the difference-form records).
__global__ void mfma_records_kernel(const double* __restrict__ xr, const double* __restrict__ wr,
                                    const int32_t* __restrict__ leaf_of_pos, const int32_t* __restrict__ begin,
                                    const int32_t* __restrict__ mgrp_off, const double* __restrict__ rctr,
                                    int64_t n, int D, const unsigned long long* __restrict__ wmax_bits,
                                    float* __restrict__ mrec, float* __restrict__ rmax2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int L = leaf_of_pos[i];
  const int idx = (int)(i - begin[L]);
  const int k2 = mfma_k2(D);
  float* g = mrec + (int64_t)(mgrp_off[L] + idx / kMG) * mfma_group_floats(D);
  const int row = idx % kMG;
  const double* c = rctr + (int64_t)L * D;
  double nrd = 0.0;  // |u_r|^2 of the float coordinates: exact squares, summed in double
  for (int d = 0; d < D; ++d) {
    const float u = (float)(xr[i * D + d] - c[d]);
    nrd += (double)u * (double)u;
    g[(d / 2) * 64 + (d % 2) * kMG + row] = -2.0f * u;
  }
  const float nr = (float)nrd;
  g[(D / 2) * 64 + (D % 2) * kMG + row] = 1.0f;
  g[((D + 1) / 2) * 64 + ((D + 1) % 2) * kMG + row] = nr;
  g[kMG * k2 + row] = (float)(wr[i] / __longlong_as_double((long long)*wmax_bits));
  atomicMax(reinterpret_cast<unsigned*>(rmax2) + L, __float_as_uint(nr));
}

__global__ void pad_counts_kernel(const int32_t* __restrict__ left, const int32_t* __restrict__ count,
                                  int n_nodes, int32_t* __restrict__ padded) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  padded[i] = left[i] < 0 ? (count[i] + kPad - 1) / kPad * kPad : 0;
}

__global__ void base_records_kernel(const double* __restrict__ xr, const double* __restrict__ wr,
                                    const int32_t* __restrict__ leaf_of_pos,
                                    const int32_t* __restrict__ begin, const int32_t* __restrict__ rec_off,
                                    const double* __restrict__ rctr, int64_t n, int D, int rs,
                                    const unsigned long long* __restrict__ wmax_bits,
                                    float* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int L = leaf_of_pos[i];
  const double* c = rctr + (int64_t)L * D;
  float* o = rec + ((int64_t)rec_off[L] + (i - begin[L])) * rs;
  for (int d = 0; d < D; ++d) o[d] = (float)(xr[i * D + d] - c[d]);
  o[D] = (float)(wr[i] / __longlong_as_double((long long)*wmax_bits));
  for (int k = D + 1; k < rs; ++k) o[k] = 0.0f;
}

// One workgroup per base group {h, Q, first, n}: key (Q, h / kHB, R), bit h % kHB.
__global__ void fuse_keys_kernel(const int4* __restrict__ grp, int ng, const int32_t* __restrict__ ent,
                                 int rbits, int hbits, unsigned long long* __restrict__ key,
                                 BaseMask* __restrict__ bit) {
  const int gi = blockIdx.x;
  if (gi >= ng) return;
  const int4 g = grp[gi];
  const unsigned long long hb = (unsigned long long)(g.x / kHB);
  const unsigned long long hi = ((unsigned long long)g.y << (hbits + rbits)) | (hb << rbits);
  const BaseMask b = (BaseMask)(1u << (g.x % kHB));
  for (int e = threadIdx.x; e < g.w; e += blockDim.x) {
    key[g.z + e] = hi | (unsigned long long)(ent[g.z + e] >> 4);
    bit[g.z + e] = b;
  }
}

struct BitOr {
  __device__ __host__ BaseMask operator()(BaseMask a, BaseMask b) const { return (BaseMask)(a | b); }
};

// Run heads (first entry of each (Q, block)) and the number of point pairs
// whose squared distance the sweep forms (one atomic per workgroup).
__global__ __launch_bounds__(1024) void run_flags_kernel(
    const unsigned long long* __restrict__ ukey, int n, int rbits, int hbits,
    const int32_t* __restrict__ qcount, const int32_t* __restrict__ rcount, int32_t* __restrict__ flag,
    unsigned long long* __restrict__ dist_evals) {
  __shared__ unsigned long long part[1024 / kW];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long pe = 0;
  if (i < n) {
    const unsigned long long k = ukey[i];
    flag[i] = (i == 0 || (k >> rbits) != (ukey[i - 1] >> rbits)) ? 1 : 0;
    const int Q = (int)(k >> (rbits + hbits));
    const int R = (int)(k & ((1ull << rbits) - 1));
    pe = (unsigned long long)qcount[Q] * (unsigned long long)rcount[R];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) pe += __shfl_xor(pe, off, kW);
  if (threadIdx.x % kW == 0) part[threadIdx.x / kW] = pe;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x / kW); ++w) t += part[w];
    if (t) atomicAdd(dist_evals, t);
  }
}

// run_start[r] = first entry of run r; run_start[nruns] = n; *nruns.
__global__ void run_scatter_kernel(const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                   int n, int32_t* __restrict__ run_start, int32_t* __restrict__ nruns) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) run_start[pos[i]] = i;
  if (i == n - 1) {
    run_start[pos[i] + flag[i]] = n;
    *nruns = pos[i] + flag[i];
  }
}

// Slices per run, and the same count for runs of several slices (whose
// slices get partial-sum slots); 0 past the last run.
__global__ void slice_counts_kernel(const int32_t* __restrict__ run_start, const int32_t* __restrict__ nruns,
                                    int n, int S, int32_t* __restrict__ nslice, int32_t* __restrict__ nmulti) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int ns = r < *nruns ? (run_start[r + 1] - run_start[r] + S - 1) / S : 0;
  nslice[r] = ns;
  nmulti[r] = ns > 1 ? ns : 0;
}

// Slices {run, first entry, end entry, partial slot (-1 when the run has a
// single slice)} and, per slot, {run, the run's first slot, its slot count}.
// counters[2] = slices, counters[3] = slots.
__global__ void slices_kernel(const int32_t* __restrict__ run_start, const int32_t* __restrict__ nruns,
                              const int32_t* __restrict__ nslice, const int32_t* __restrict__ sstart,
                              const int32_t* __restrict__ nmulti, const int32_t* __restrict__ mstart, int S,
                              int max_slots, int4* __restrict__ slices, int4* __restrict__ slots,
                              int32_t* __restrict__ counters) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = *nruns;
  if (r >= nr) return;
  const int e0 = run_start[r], e1 = run_start[r + 1], ns = nslice[r], s0 = sstart[r];
  const int m0 = mstart[r];
  for (int j = 0; j < ns; ++j) {
    const int a = e0 + j * S;
    const int slot = ns > 1 && m0 + j < max_slots ? m0 + j : -1;
    slices[s0 + j] = make_int4(r, a, min(e1, a + S), slot);
    if (slot >= 0) slots[slot] = make_int4(r, m0, ns, 0);
  }
  if (r == nr - 1) {
    counters[2] = s0 + ns;
    counters[3] = m0 + nmulti[r];
  }
}

// Estimated issue cost of each slice, as a descending sort key (capped to
// 16 bits), and the identity order: per entry, its padded reference count
// times (2 D + 4 per bandwidth of its mask) plus a fixed per-entry overhead.
// Units are then taken heaviest first, so that the units still running when
// the queue runs dry are light ones.
__global__ void slice_cost_kernel(const int4* __restrict__ slices, int n_slices,
                                  const unsigned long long* __restrict__ ukey,
                                  const BaseMask* __restrict__ umask, int rbits, const int32_t* __restrict__ rcount,
                                  int D, uint32_t* __restrict__ key, int32_t* __restrict__ idx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_slices) return;
  const int4 sd = slices[i];
  const unsigned long long rmask = (1ull << rbits) - 1;
  uint64_t c = 0;
  for (int e = sd.y; e < sd.z; ++e) {
    const int rnp = (rcount[(int)(ukey[e] & rmask)] + kPad - 1) / kPad * kPad;
    c += (uint64_t)rnp * (uint64_t)(2 * D + 4 * __builtin_popcount(umask[e])) + kEntryCost;
  }
  c >>= 4;
  key[i] = (uint32_t)(c < 65535 ? c : 65535);
  idx[i] = i;
}

// Sixteen floats read by one scalar load when the address is wave-uniform.
typedef float f16v __attribute__((ext_vector_type(16), aligned(16)));

// Sweep of one reference leaf for NA bandwidths: for every record r,
//   part[j] += w_r exp2(-(|u_q - u_r|^2 - t2) shc[j]),  j < NA,
// with t2 the lane's shift in squared-distance units (the sum is scaled by
// 2^(t2 shc[j]), which the caller takes out exactly in double).
// p: the leaf's padded records, nb batches of BR records of RS floats; a
// batch is read as whole 16-float vectors (up to 15 floats past the batch,
// inside the record array's tail).
template <int D, int NA, int RS, int BR>
__device__ __forceinline__ void sweep(const float* __restrict__ p, int nb, const float* uq,
                                      const float* shc, float t2, float* part) {
  constexpr int NF = RS * BR;
  constexpr int NV = (NF + 15) / 16;
  for (int b = 0; b < nb; ++b, p += NF) {
    f16v v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = *reinterpret_cast<const f16v*>(p + 16 * i);
#pragma unroll
    for (int j = 0; j < BR; ++j) {
      float d2 = 0.0f;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const float dd = uq[d] - v[(j * RS + d) / 16][(j * RS + d) % 16];
        d2 = fmaf(dd, dd, d2);
      }
      const float wr = v[(j * RS + D) / 16][(j * RS + D) % 16];
      const float e = d2 - t2;
#pragma unroll
      for (int a = 0; a < NA; ++a) part[a] = fmaf(wr, __builtin_amdgcn_exp2f(-e * shc[a]), part[a]);
    }
  }
}

// Smallest |u_q - u_r|^2 over the records of a leaf (padding records are far
// away and never the smallest).
template <int D, int RS, int BR>
__device__ __forceinline__ float sweep_min(const float* __restrict__ p, int nb, const float* uq) {
  constexpr int NF = RS * BR;
  constexpr int NV = (NF + 15) / 16;
  float m2 = INFINITY;
  for (int b = 0; b < nb; ++b, p += NF) {
    f16v v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = *reinterpret_cast<const f16v*>(p + 16 * i);
#pragma unroll
    for (int j = 0; j < BR; ++j) {
      float d2 = 0.0f;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const float dd = uq[d] - v[(j * RS + d) / 16][(j * RS + d) % 16];
        d2 = fmaf(dd, dd, d2);
      }
      m2 = fminf(m2, d2);
    }
  }
  return m2;
}

// Any D: one record at a time.
template <int NA>
__device__ __forceinline__ void sweep_any(const float* __restrict__ p, int n, int D, int rs,
                                          const float* uq, const float* shc, float t2, float* part) {
  for (int r = 0; r < n; ++r, p += rs) {
    float d2 = 0.0f;
    for (int d = 0; d < D; ++d) {
      const float dd = uq[d] - p[d];
      d2 = fmaf(dd, dd, d2);
    }
    const float wr = p[D];
    const float e = d2 - t2;
#pragma unroll
    for (int a = 0; a < NA; ++a) part[a] = fmaf(wr, __builtin_amdgcn_exp2f(-e * shc[a]), part[a]);
  }
}

__device__ __forceinline__ float sweep_min_any(const float* __restrict__ p, int n, int D, int rs,
                                               const float* uq) {
  float m2 = INFINITY;
  for (int r = 0; r < n; ++r, p += rs) {
    float d2 = 0.0f;
    for (int d = 0; d < D; ++d) {
      const float dd = uq[d] - p[d];
      d2 = fmaf(dd, dd, d2);
    }
    m2 = fminf(m2, d2);
  }
  return m2;
}

template <int DT>
__device__ __forceinline__ float sweep_leaf_min(const float* __restrict__ rec, int rs, int D, int rn_padded,
                                                const float* uq) {
  if constexpr (DT > 0) {
    constexpr int RS = (DT + 4) / 4 * 4;
    constexpr int BR = RS == 4 ? 4 : RS == 8 ? 2 : 1;
    return sweep_min<DT, RS, BR>(rec, rn_padded / BR, uq);
  } else {
    return sweep_min_any(rec, rn_padded, D, rs, uq);
  }
}

template <int DT, int NA>
__device__ __forceinline__ void sweep_leaf(const float* __restrict__ rec, int rs, int D, int rn_padded,
                                           const float* uq, const float* shc, float t2, float* part) {
  if constexpr (DT > 0) {
    constexpr int RS = (DT + 4) / 4 * 4;
    constexpr int BR = RS == 4 ? 4 : RS == 8 ? 2 : 1;
    sweep<DT, NA, RS, BR>(rec, rn_padded / BR, uq, shc, t2, part);
  } else {
    sweep_any<NA>(rec, rn_padded, D, rs, uq, shc, t2, part);
  }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Sweep of one reference leaf with squared distances from the MFMA norm
// expansion, for NA bandwidths and the wave's 64 queries in two halves of 32,
// one half after the other: in half s, lane l takes query (l % 32) + 32 s and
// the references of rows 8 j + 4 (l / 32) + i (j, i < 4) of each 32-reference
// group, for which one v_mfma_f32_32x32x2f32 per pair of augmented
// coordinates leaves |u_q - u_r|^2 - T_q in its 16 accumulator registers (A:
// the group's records (-2 u_r, 1, |u_r|^2), B: the queries' (u_q,
// |u_q|^2 - T_q, 1), with T_q the query's squared distance to the leaf's box,
// so that every exponent -s_h (|u_q - u_r|^2 - T_q) is <= 0 up to rounding).
// At the end of a half the two lanes of a query add their partial sums; a
// bandwidth whose sum is below 2^-60 for any of the half's queries is left to
// the rescue (bit j of the returned mask, shifted by 16 for the second half),
// and the query's own lane adds the others to its accumulators acc[k * 64]
// (k: the block index of the j-th bandwidth of `bits`), unscaled by
// 2^(T_q s_h) in double.  Only one half's NA sums are live at a time (the
// group's records are read again for the second half, from cache).
template <int D, int NA>
__device__ __forceinline__ unsigned mfma_sweep(const float* __restrict__ mg, int ngroups, int nsub,
                                               const float* uq, float nqt, const float* shc, unsigned bits,
                                               double* acc, float tq, int qrem) {
  constexpr int K2 = mfma_k2(D), KM = K2 / 2, GF = mfma_group_floats(D);
  const int lane = threadIdx.x & (kW - 1);
  const int half = lane >> 5;
  float v[K2];
#pragma unroll
  for (int k = 0; k < K2; ++k) v[k] = k < D ? uq[k < D ? k : 0] : k == D ? nqt : k == D + 1 ? 1.0f : 0.0f;
  unsigned lows = 0;
  for (int s = 0; s < nsub; ++s) {
    const int src = (lane & 31) + 32 * s;
    float bq[KM];
#pragma unroll
    for (int m = 0; m < KM; ++m) {
      const float e0 = __shfl(v[2 * m], src, kW);
      const float e1 = __shfl(v[2 * m + 1], src, kW);
      bq[m] = half ? e1 : e0;
    }
    float p[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) p[j] = 0.0f;
    const float* g = mg;
    for (int gi = 0; gi < ngroups; ++gi, g += GF) {
      float a[KM];
#pragma unroll
      for (int m = 0; m < KM; ++m) a[m] = g[m * 64 + lane];
      float4 w4[4];
#pragma unroll
      for (int j4 = 0; j4 < 4; ++j4)
        w4[j4] = *reinterpret_cast<const float4*>(g + kMG * K2 + 8 * j4 + 4 * half);
      f32x16 c = {};
#pragma unroll
      for (int m = 0; m < KM; ++m) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m], bq[m], c, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float wr = w4[i / 4][i % 4];
#pragma unroll
        for (int j = 0; j < NA; ++j) p[j] = fmaf(wr, __builtin_amdgcn_exp2f(-c[i] * shc[j]), p[j]);
      }
    }
    unsigned lo = 0;
    const bool act = (lane & 31) + 32 * s < qrem;  // the half's query of this lane exists
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      p[j] += __shfl_xor(p[j], 32, kW);
      if (__any(act && p[j] < 0x1p-60f)) lo |= 1u << j;
    }
    if (half == s) {
      unsigned mm = bits;
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        const int k = __builtin_ctz(mm);
        mm &= mm - 1;
        if ((lo >> j) & 1u) continue;
        const double sc = (double)tq * (double)shc[j];
        const double fi = floor(sc);
        acc[k * kW] += ldexp((double)(p[j] * __builtin_amdgcn_exp2f((float)(fi - sc))), -(int)fi);
      }
    }
    lows |= lo << (16 * s);
  }
  return lows;
}

// The NA = 1..kHB specialisations: each spends exactly one exp2 per needed
// (point pair, bandwidth).
#define GS_NA_CASES(F)                                                                              \
  switch (na) {                                                                                     \
    case 1: F(1); break;   case 2: F(2); break;   case 3: F(3); break;   case 4: F(4); break;       \
    case 5: F(5); break;   case 6: F(6); break;   case 7: F(7); break;   case 8: F(8); break;       \
    case 9: F(9); break;   case 10: F(10); break; case 11: F(11); break; case 12: F(12); break;     \
    case 13: F(13); break; case 14: F(14); break; case 15: F(15); break; default: F(16); break;      \
  }
static_assert(kHB == 16, "GS_NA_CASES lists kHB cases");

template <int DT>
__device__ __forceinline__ unsigned mfma_sweep_leaf(int na, const float* __restrict__ mg, int ngroups, int nsub,
                                                    const float* uq, float nqt, const float* shc, unsigned bits,
                                                    double* acc, float tq, int qrem) {
  unsigned lows = 0;
#define GS_MFMA_CASE(NA) lows = mfma_sweep<DT, NA>(mg, ngroups, nsub, uq, nqt, shc, bits, acc, tq, qrem)
  GS_NA_CASES(GS_MFMA_CASE)
#undef GS_MFMA_CASE
  return lows;
}

template <int DT>
__device__ __forceinline__ void sweep_leaf_na(int na, const float* __restrict__ rp, int rs, int D, int rnp,
                                              const float* uq, const float* shc, float t2, float* part) {
#define GS_SWEEP_CASE(NA) sweep_leaf<DT, NA>(rp, rs, D, rnp, uq, shc, t2, part)
  GS_NA_CASES(GS_SWEEP_CASE)
#undef GS_SWEEP_CASE
}

// Persistent waves (four per SIMD: the MFMA sweeps use up to 128 registers,
// and four already keep the VALU busy) take work units from a queue counter until
// none is left, heaviest slices first (slice_cost_kernel): unit u is query batch
// u % QB (64 queries) of slice u / QB, QB = qmax / 64.  There are several
// units per wave, so a SIMD whose units were light takes more of them and
// all finish together; the two batches of a slice are taken back to back and
// read the same reference leaves.  The reference records (a few MB) stay in
// every XCD's L2, so the order in which units meet XCDs does not matter.
//
// The instruction arbiter serves the oldest wave of a SIMD first, so without
// help the youngest waves hold their first unit for most of the sweep and
// finish it alone at the end.  A wave therefore raises its priority by one
// step for every kAgeStep of real time (100 MHz clock) that its current unit
// has taken, and drops back to 0 when it takes the next unit: a starved unit
// catches up instead of becoming the tail.  Workgroups hold kBaseWaves
// independent waves (no LDS, no barrier).
template <int DT>
__global__ __launch_bounds__(kW * kBaseWaves) __attribute__((amdgpu_waves_per_eu(4))) void base_fused_kernel(
    const int4* __restrict__ slices, const int32_t* __restrict__ order, int n_slices,
    const int32_t* __restrict__ run_start, const unsigned long long* __restrict__ ukey,
    const BaseMask* __restrict__ umask, int rbits, int hbits, int hc0, int hc1, NodeView qt, NodeView rt,
    const int32_t* __restrict__ rec_off, const double* __restrict__ xq_perm, const float* __restrict__ rec,
    const int32_t* __restrict__ mgrp_off, const float* __restrict__ mrec, const float* __restrict__ rmax2,
    int Drt, int rs_rt, const float* __restrict__ s2, const unsigned long long* __restrict__ wmax_bits,
    int Mq, int qmax, double* __restrict__ partial, double* __restrict__ gx,
    int32_t* __restrict__ queue, unsigned long long* __restrict__ mfma_evals) {
  constexpr int DC = DT > 0 ? DT : kMaxD;
  const int D = DT > 0 ? DT : Drt;
  const int rs = DT > 0 ? (DT + 4) / 4 * 4 : rs_rt;
  const int QB = qmax / kW;
  const int n_units = n_slices * QB;
  const int lane = threadIdx.x & (kW - 1);
  __shared__ double acc_lds[kBaseWaves * kHB * kW];
  unsigned long long mfma_pairs = 0;  // point-pair evaluations from MFMA distances (uniform)
  for (;;) {
  int grab = 0;
  if (lane == 0) grab = atomicAdd(queue, 1);
  const int u = __builtin_amdgcn_readfirstlane(grab);
  if (u >= n_units) break;
  __builtin_amdgcn_s_setprio(0);
  const uint64_t t_unit = __builtin_amdgcn_s_memrealtime();
  int prio = 0;
  const int si = u / QB;
  const int base = (u - si * QB) * kW;
  const int4 sd = slices[order[si]];
  const unsigned long long k0 = ukey[run_start[sd.x]];
  const int Q = (int)(k0 >> (hbits + rbits));
  const int h0 = (int)((k0 >> rbits) & ((1ull << hbits) - 1)) * kHB;
  const unsigned long long rmask = (1ull << rbits) - 1;
  const int qb = qt.begin[Q], qn = qt.count[Q];
  if (base < qn) {
    const bool active = base + lane < qn;
    const int qpos = qb + base + (active ? lane : 0);
    // the unit's sums per bandwidth live in LDS, not registers: they are
    // touched once per entry, and registers are what the sweeps need
    double* acc = acc_lds + (threadIdx.x / kW) * kHB * kW + lane;
#pragma unroll
    for (int k = 0; k < kHB; ++k) acc[k * kW] = 0.0;
    for (int e = sd.y; e < sd.z; ++e) {
      if (prio < 3) {
        const uint64_t age = __builtin_amdgcn_s_memrealtime() - t_unit;
        if (age > (uint64_t)(prio + 1) * kAgeStep) {
          ++prio;
          if (prio == 1) __builtin_amdgcn_s_setprio(1);
          else if (prio == 2) __builtin_amdgcn_s_setprio(2);
          else __builtin_amdgcn_s_setprio(3);
        }
      }
      const int R = (int)(ukey[e] & rmask);
      const unsigned m = umask[e];
      const double* cR = rt.ctr + (int64_t)R * D;
      const double* lR = rt.lo + (int64_t)R * D;
      const double* hR = rt.hi + (int64_t)R * D;
      // the query's coordinates are read for every entry (from cache) rather
      // than held in registers across the unit
      double xq[DC];
#pragma unroll
      for (int d = 0; d < DC; ++d)
        if (d < D) xq[d] = xq_perm[(int64_t)qpos * D + d];
      float uq[DC];
      double box2 = 0.0;
#pragma unroll
      for (int d = 0; d < DC; ++d) {
        if (d < D) {
          uq[d] = (float)(xq[d] - cR[d]);
          double gap = lR[d] - xq[d];
          const double o = xq[d] - hR[d];
          gap = o > gap ? o : gap;
          gap = gap > 0.0 ? gap : 0.0;
          box2 += gap * gap;
        }
      }
      // Bandwidths whose squared distances may come from the MFMA norm
      // expansion (file comment): the expansion's rounding error is at most
      // kMfmaErrC 2^-24 (|u_q| + |u_r|)^2, which moves a term's exponent by at
      // most that times s_h; a bandwidth is admitted when the resulting
      // relative error of every term is below kMfmaTau.
      unsigned safe = 0;
      float nqt = 0.0f;              // |u_q|^2 - T_q, the query's augmented coordinate
      const float tq = (float)box2;  // the box shift T_q of the MFMA path
      if (mfma_dim(DT) && mrec != nullptr) {
        double nqd = 0.0;  // |u_q|^2 of the float coordinates: exact squares, summed in double
#pragma unroll
        for (int d = 0; d < DC; ++d)
          if (d < D) nqd += (double)uq[d] * (double)uq[d];
        nqt = (float)(nqd - (double)tq);
        float mx = (float)nqd;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, kW));
        const float rr = sqrtf(rmax2[R]) + sqrtf(mx);
        const float bnd = (float)kMfmaErrC<DT> * 0x1p-24f * 0.6931472f * 1.0001f * (rr * rr);
#pragma unroll
        for (int k = 0; k < kHB; ++k)
          if (((m >> k) & 1u) && bnd * s2[h0 + k] <= kMfmaTau) safe |= 1u << k;
        safe = __builtin_amdgcn_readfirstlane(safe);
      }
      const float* rp = rec + (int64_t)rec_off[R] * rs;
      const int rnp = (rt.count[R] + kPad - 1) / kPad * kPad;
      for (int sub = 0; sub < 2; ++sub) {
        const unsigned bits = sub == 0 ? safe : (m & ~safe);
        if (bits == 0) continue;
        const bool use_mfma = sub == 0;
        // Compact the subset's bandwidths: j-th set bit -> shc[j] (uniform).
        const int na = __builtin_popcount(bits);
        float shc[kHB], part[kHB];
        {
          unsigned mm = bits;
#pragma unroll
          for (int j = 0; j < kHB; ++j) {
            const int k = mm ? __builtin_ctz(mm) : 0;
            mm &= mm - 1;
            shc[j] = s2[h0 + k];
            part[j] = 0.0f;
          }
        }
        if (use_mfma) mfma_pairs += (unsigned long long)na * (unsigned long long)rt.count[R] *
                                    (unsigned long long)(qn - base < kW ? qn - base : kW);
        // Adds the sums of the subset's j-th bandwidths selected by jmask to
        // the unit's accumulators, unscaled in double: a sweep with shift t2
        // (squared-distance units; T_q folded into the MFMA operands is the
        // same shift) leaves its terms scaled by 2^(t2 s_h), and t2 s_h is
        // formed exactly in double.
        auto accumulate = [&](unsigned jmask, float t2) {
          unsigned mm = bits;
          // left rolled: once per entry and bandwidth, and 16 unrolled copies
          // of its double arithmetic at each call measured slower
          for (int j = 0; j < kHB; ++j) {
            if (mm == 0) break;
            const int k = __builtin_ctz(mm);
            mm &= mm - 1;
            if (!((jmask >> j) & 1u)) continue;
            const double sc = (double)t2 * (double)shc[j];
            const double fi = floor(sc);
            acc[k * kW] += ldexp((double)(part[j] * __builtin_amdgcn_exp2f((float)(fi - sc))), -(int)fi);
          }
        };
        // Rescue (file comment): a bandwidth whose sum is below 2^-60 on any
        // active lane (of a half, on the MFMA path) takes its shift from the
        // lane's smallest distance, and the wave sweeps the leaf again
        // (difference form); the other bandwidths keep their first sweep, so
        // a bandwidth's result does not depend on which other bandwidths share
        // the entry.
        auto rescue = [&](unsigned lanelow) {
          const float m2 = sweep_leaf_min<DT>(rp, rs, D, rnp, uq);
          const float t2 = fmaxf(tq, m2);
#pragma unroll
          for (int j = 0; j < kHB; ++j) part[j] = 0.0f;
          sweep_leaf_na<DT>(na, rp, rs, D, rnp, uq, shc, t2, part);
          accumulate(lanelow, t2);
        };
        if (use_mfma) {
          if constexpr (mfma_dim(DT)) {
            const int qrem = qn - base;
            const unsigned lows =
                mfma_sweep_leaf<DT>(na, mrec + (int64_t)mgrp_off[R] * mfma_group_floats(DT),
                                    (rt.count[R] + kMG - 1) / kMG, qrem > kMG ? 2 : 1, uq, nqt, shc, bits,
                                    acc, tq, qrem);
            if (lows != 0) rescue(lane >= 32 ? lows >> 16 : lows & 0xffffu);
          }
        } else {
          sweep_leaf_na<DT>(na, rp, rs, D, rnp, uq, shc, tq, part);
          unsigned low = 0;
#pragma unroll
          for (int j = 0; j < kHB; ++j)
            if (j < na && __any(active && part[j] < 0x1p-60f)) low |= 1u << j;
          accumulate(~low, tq);
          if (low != 0) rescue(low);
        }
      }
    }
    if (active) {
      if (sd.w < 0) {
        const double wscale = __longlong_as_double((long long)*wmax_bits);
#pragma unroll
        for (int k = 0; k < kHB; ++k)
          if (h0 + k >= hc0 && h0 + k < hc1) gx[(int64_t)(h0 + k) * Mq + qpos] = acc[k * kW] * wscale;
      } else {
        double* pp = partial + (int64_t)sd.w * kHB * qmax + base + lane;
#pragma unroll
        for (int k = 0; k < kHB; ++k) pp[(int64_t)k * qmax] = acc[k * kW];
      }
    }
  }
  }  // next slice
  if (lane == 0 && mfma_pairs) atomicAdd(mfma_evals, mfma_pairs);
}

// Runs of several slices: gx = sum of the slices' partials in slice order.
// One workgroup per partial slot; only a run's first slot does the work, one
// thread per (bandwidth, query) of the run's query leaf.
__global__ __launch_bounds__(kReduceThreads) void base_reduce_kernel(
    const int4* __restrict__ slots, int n_slots,
    const int32_t* __restrict__ run_start, const unsigned long long* __restrict__ ukey, int rbits, int hbits,
    int hc0, int hc1, NodeView qt, const unsigned long long* __restrict__ wmax_bits, int Mq, int qmax,
    const double* __restrict__ partial, double* __restrict__ gx) {
  const int sl = blockIdx.x;
  if (sl >= n_slots) return;
  const int4 info = slots[sl];
  if (info.y != sl) return;
  const int ns = info.z;
  const unsigned long long k0 = ukey[run_start[info.x]];
  const int Q = (int)(k0 >> (hbits + rbits));
  const int h0 = (int)((k0 >> rbits) & ((1ull << hbits) - 1)) * kHB;
  const int qb = qt.begin[Q], qn = qt.count[Q];
  const double wscale = __longlong_as_double((long long)*wmax_bits);
  const int nj = min(ns, n_slots - sl);
  for (int i = threadIdx.x; i < kHB * qn; i += kReduceThreads) {
    const int k = i / qn, q = i - k * qn;
    if (h0 + k < hc0 || h0 + k >= hc1) continue;
    const double* pp = partial + ((int64_t)sl * kHB + k) * qmax + q;
    double v = 0.0;
    for (int j = 0; j < nj; ++j) v += pp[(int64_t)j * kHB * qmax];
    gx[(int64_t)(h0 + k) * Mq + qb + q] = v * wscale;
  }
}

int bits_for(int64_t n) {
  int b = 1;
  while ((1ll << b) < n) ++b;
  return b;
}

template <int DT>
void launch_fused_t(const BaseFusedArgs& a, const BaseFusedPlan& p, hipStream_t s) {
  const int64_t waves = std::min<int64_t>((int64_t)p.n_slices * (p.qmax / kW), kResidentWaves);
  const int nb = (int)ceil_div(waves, kBaseWaves);
  (void)hipMemsetAsync(a.counters + 4, 0, sizeof(int32_t), s);
  hipLaunchKernelGGL((base_fused_kernel<DT>), dim3((unsigned)nb), dim3(kW * kBaseWaves), 0, s, a.slices, a.mpos,
                     p.n_slices,
                     a.run_start, a.ukey, a.umask, p.rbits, p.hbits, a.hc0, a.hc1, a.qt,
                     a.rt, a.rec_off, a.xq_perm, a.rec, a.mgrp_off, a.mrec, a.rmax2, a.D, base_record_stride(a.D),
                     a.s2, a.wmax_bits, a.Mq, p.qmax, a.partial, a.gx, a.counters + 4, a.mfma_evals);
}

}  // namespace

int base_record_stride(int D) { return (D + 1 + 3) / 4 * 4; }

int64_t base_records_capacity(int64_t n_points, int n_nodes) {
  // padding of at most kPad - 1 per leaf, plus a tail for the 16-float reads
  return n_points + (int64_t)(kPad - 1) * n_nodes + 16;
}

size_t base_records_temp_bytes(int n_nodes) {
  size_t b = 0;
  (void)rocprim::exclusive_scan((void*)nullptr, b, (const int32_t*)nullptr, (int32_t*)nullptr, 0,
                                (size_t)n_nodes, rocprim::plus<int32_t>());
  return b;
}

bool base_uses_mfma(int D) { return D == 2 || D == 3 || D == 4 || D == 5 || D == 8 || D == 16; }

int64_t base_mfma_groups_capacity(int64_t n_points, int n_nodes) { return n_points / kMG + n_nodes + 1; }

int base_mfma_group_floats(int D) { return mfma_group_floats(D); }

hipError_t launch_base_records(const BaseRecordsArgs& a, hipStream_t s) {
  if (a.mrec) {
    // MFMA records: padding everywhere, group offsets per leaf, then the points
    const int64_t mf = a.mgroups_capacity * mfma_group_floats(a.D);
    hipLaunchKernelGGL(mfma_pad_kernel, dim3((unsigned)ceil_div(mf, 256)), dim3(256), 0, s, a.mrec, mf, a.D);
    hipLaunchKernelGGL(mfma_groups_kernel, dim3((unsigned)ceil_div(a.n_nodes, 256)), dim3(256), 0, s, a.left,
                       a.count, a.n_nodes, a.padded, a.rmax2);
    size_t mbytes = a.temp_bytes;
    hipError_t me = rocprim::exclusive_scan(a.temp, mbytes, a.padded, a.mgrp_off, 0, (size_t)a.n_nodes,
                                            rocprim::plus<int32_t>(), s);
    if (me != hipSuccess) return me;
    hipLaunchKernelGGL(mfma_records_kernel, dim3((unsigned)ceil_div(a.n, 256)), dim3(256), 0, s, a.xr_perm,
                       a.wr_perm, a.leaf_of_pos, a.begin, a.mgrp_off, a.rctr, a.n, a.D, a.wmax_bits, a.mrec,
                       a.rmax2);
    me = hipGetLastError();
    if (me != hipSuccess) return me;
  }
  const int64_t n_floats = a.rec_capacity * base_record_stride(a.D);
  hipLaunchKernelGGL(pad_records_kernel, dim3((unsigned)ceil_div(n_floats, 256)), dim3(256), 0, s, a.rec, n_floats,
                     a.D, base_record_stride(a.D));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pad_counts_kernel, dim3((unsigned)ceil_div(a.n_nodes, 256)), dim3(256), 0, s, a.left,
                     a.count, a.n_nodes, a.padded);
  size_t bytes = a.temp_bytes;
  e = rocprim::exclusive_scan(a.temp, bytes, a.padded, a.rec_off, 0, (size_t)a.n_nodes,
                              rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(base_records_kernel, dim3((unsigned)ceil_div(a.n, 256)), dim3(256), 0, s, a.xr_perm,
                     a.wr_perm, a.leaf_of_pos, a.begin, a.rec_off, a.rctr, a.n, a.D, base_record_stride(a.D),
                     a.wmax_bits, a.rec);
  return hipGetLastError();
}

size_t base_fused_temp_bytes(int64_t n) {
  size_t b1 = 0, b2 = 0, b3 = 0;
  (void)rocprim::radix_sort_pairs((void*)nullptr, b1, (const unsigned long long*)nullptr,
                                  (unsigned long long*)nullptr, (const BaseMask*)nullptr,
                                  (BaseMask*)nullptr, (size_t)n, 0, 64);
  (void)rocprim::reduce_by_key((void*)nullptr, b2, (const unsigned long long*)nullptr,
                               (const BaseMask*)nullptr, (size_t)n, (unsigned long long*)nullptr,
                               (BaseMask*)nullptr, (int32_t*)nullptr, BitOr(),
                               rocprim::equal_to<unsigned long long>());
  (void)rocprim::exclusive_scan((void*)nullptr, b3, (const int32_t*)nullptr, (int32_t*)nullptr, 0,
                                (size_t)n, rocprim::plus<int32_t>());
  size_t b4 = 0;
  (void)rocprim::radix_sort_pairs_desc((void*)nullptr, b4, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                       (const int32_t*)nullptr, (int32_t*)nullptr, (size_t)n, 0, 16);
  return std::max(std::max(b1, b2), std::max(b3, b4));
}

// Partial-sum slots of one call: 4 * 16384 * 64 / qmax, so the partials take
// 4 * 16384 * 64 * kHB doubles (512 MiB) whatever the leaf size.
int base_partial_slots(int max_leaf) {
  const int qmax = (int)ceil_div(std::max(1, max_leaf), kW) * kW;
  return 4 * 16384 * kW / qmax;
}

int64_t base_partial_doubles(int max_leaf) {
  const int qmax = (int)ceil_div(std::max(1, max_leaf), kW) * kW;
  return (int64_t)base_partial_slots(max_leaf) * kHB * qmax;
}

// Entries per slice: about base_partial_slots / 2 slices in all, at least 8
// entries each; with a slice's query batches that is 32768 work units, four
// per resident wave, whatever the leaf size.  A run of len > S entries
// has ceil(len / S) < 2 len / S slices, so the runs of several slices hold
// fewer than 2 n_unique / S <= base_partial_slots slices.
int base_slice_entries(int64_t n_unique, int max_leaf) {
  const int64_t target = base_partial_slots(max_leaf) / 2;
  return (int)std::max<int64_t>(8, (n_unique + target - 1) / target);
}

int64_t base_max_slices(int64_t n_entries) {
  // runs <= entries, and slices <= runs + entries / S with S >= 8
  return n_entries + n_entries / 8 + 1;
}

hipError_t plan_base_fused(const BaseFusedArgs& a, BaseFusedPlan* p, hipStream_t s) {
  p->n_slices = 0;
  const int64_t n = a.n_entries;
  if (n == 0 || a.n_groups == 0) return hipSuccess;
  p->rbits = bits_for(a.n_rnodes + 1);
  p->hbits = bits_for(a.n_hblocks + 1);
  p->qmax = (int)ceil_div(a.max_leaf, kW) * kW;
  const int qbits = bits_for(a.n_qnodes + 1);
  if (p->rbits + p->hbits + qbits > 63 || n > INT32_MAX / 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fuse_keys_kernel, dim3((unsigned)a.n_groups), dim3(64), 0, s, a.grp, a.n_groups,
                     a.ent, p->rbits, p->hbits, a.key, a.bit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t bytes = a.temp_bytes;
  e = rocprim::radix_sort_pairs(a.temp, bytes, a.key, a.key_sorted, a.bit, a.bit_sorted, (size_t)n, 0,
                                p->rbits + p->hbits + qbits, s);
  if (e != hipSuccess) return e;
  bytes = a.temp_bytes;
  e = rocprim::reduce_by_key(a.temp, bytes, a.key_sorted, a.bit_sorted, (size_t)n, a.ukey, a.umask,
                             a.counters, BitOr(), rocprim::equal_to<unsigned long long>(), s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(a.host_counters, a.counters, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int32_t nu = a.host_counters[0];
  if (nu <= 0 || nu > n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(run_flags_kernel, dim3((unsigned)ceil_div(nu, 1024)), dim3(1024), 0, s, a.ukey, nu,
                     p->rbits, p->hbits, a.qt.count, a.rt.count, a.flag, a.dist_evals);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  bytes = a.temp_bytes;
  e = rocprim::exclusive_scan(a.temp, bytes, a.flag, a.pos, 0, (size_t)nu, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(run_scatter_kernel, dim3((unsigned)ceil_div(nu, 256)), dim3(256), 0, s, a.flag,
                     a.pos, nu, a.run_start, a.counters + 1);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // Slices: counts per run into flag and mflag, their exclusive scans into
  // pos and mpos (runs <= nu, counts past the last run are 0).
  const int S = base_slice_entries(nu, a.max_leaf);
  hipLaunchKernelGGL(slice_counts_kernel, dim3((unsigned)ceil_div(nu, 256)), dim3(256), 0, s, a.run_start,
                     a.counters + 1, nu, S, a.flag, a.mflag);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  bytes = a.temp_bytes;
  e = rocprim::exclusive_scan(a.temp, bytes, a.flag, a.pos, 0, (size_t)nu, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  bytes = a.temp_bytes;
  e = rocprim::exclusive_scan(a.temp, bytes, a.mflag, a.mpos, 0, (size_t)nu, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  p->max_slots = base_partial_slots(a.max_leaf);
  hipLaunchKernelGGL(slices_kernel, dim3((unsigned)ceil_div(nu, 256)), dim3(256), 0, s, a.run_start,
                     a.counters + 1, a.flag, a.pos, a.mflag, a.mpos, S, p->max_slots, a.slices, a.slots,
                     a.counters);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  p->slice_entries = S;
  e = hipMemcpyAsync(a.host_counters, a.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int32_t* cnt = a.host_counters;
  // slices <= nu (a slice holds at least one entry); slots < 2 nu / S <= max_slots
  if (cnt[2] <= 0 || cnt[2] > nu || cnt[3] < 0 || cnt[3] > p->max_slots)
    return hipErrorInvalidValue;
  // work units (slice, query batch) are counted in int32
  if ((int64_t)cnt[2] * (p->qmax / kW) > INT32_MAX - kResidentWaves) return hipErrorInvalidValue;
  p->n_slices = cnt[2];
  p->n_slots = cnt[3];
  // Slice order, heaviest first, into mpos (slices <= unique entries, so the
  // entry-sized scratch arrays hold it; flag, pos and mflag are free now).
  uint32_t* ckey = reinterpret_cast<uint32_t*>(a.flag);
  uint32_t* ckey_sorted = reinterpret_cast<uint32_t*>(a.mflag);
  hipLaunchKernelGGL(slice_cost_kernel, dim3((unsigned)ceil_div(p->n_slices, 256)), dim3(256), 0, s, a.slices,
                     p->n_slices, a.ukey, a.umask, p->rbits, a.rt.count, a.D, ckey, a.pos);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  bytes = a.temp_bytes;
  e = rocprim::radix_sort_pairs_desc(a.temp, bytes, ckey, ckey_sorted, a.pos, a.mpos, (size_t)p->n_slices, 0, 16,
                                     s);
  if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_base_fused(const BaseFusedArgs& a, const BaseFusedPlan& p, hipStream_t s) {
  if (p.n_slices == 0) return hipSuccess;
  switch (a.D) {
    case 1: launch_fused_t<1>(a, p, s); break;
    case 2: launch_fused_t<2>(a, p, s); break;
    case 3: launch_fused_t<3>(a, p, s); break;
    case 4: launch_fused_t<4>(a, p, s); break;
    case 5: launch_fused_t<5>(a, p, s); break;
    case 8: launch_fused_t<8>(a, p, s); break;
    case 16: launch_fused_t<16>(a, p, s); break;
    default: launch_fused_t<0>(a, p, s); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.n_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(base_reduce_kernel, dim3((unsigned)p.n_slots), dim3(kReduceThreads), 0, s, a.slots, p.n_slots,
                     a.run_start, a.ukey, p.rbits, p.hbits, a.hc0, a.hc1, a.qt, a.wmax_bits,
                     a.Mq, p.qmax, a.partial, a.gx);
  return hipGetLastError();
}

}  // namespace gs
