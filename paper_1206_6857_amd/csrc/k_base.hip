// Exhaustive base cases of the dual-tree traversal (DITOBase, Figure 7),
// fused over bandwidths:
//     gx[h][q] = sum over base pairs (Q, R) of h, r in R:  w_r exp(-|x_q - x_r|^2 / 2h^2),
// for q in the leaf Q.
//
// The traversal records base pairs per (h, Q).  The same leaf pair is usually
// a base case for several neighbouring bandwidths, and |x_q - x_r|^2 does not
// depend on h, so the entries are regrouped by (Q, block of 8 bandwidths, R)
// with an 8-bit mask of the block's bandwidths that need the pair: a radix sort
// of (Q, block, R) keys, then an OR reduction by key.  A run is the set of
// regrouped entries of one (Q, block).  One workgroup of kWaves waves handles
// one run: lanes hold the points of Q, the run's entries are dealt round-robin
// to the waves, and every point pair's squared distance feeds one exp2 per
// bandwidth of the entry's mask.  Reference points are read with wave-uniform
// addresses (scalar loads, no LDS staging).  The per-wave partials are summed in
// wave order, so every gx[h][q] is written once and the result is
// deterministic.
//
// Precision: reference coordinates are stored relative to their leaf centre
// in float (u_r = x_r - c_R); each lane forms u_q = x_q - c_R in double before
// rounding to float, so u_q - u_r is accurate to ~2^-24 of the pair's extent.
// Every term of a leaf pair is scaled by exp(+d_box^2 / 2h^2), where d_box is
// the distance from x_q to R's bounding box (a lower bound of |x_q - x_r|, so
// each scaled term is <= 1 and far pairs stay out of the float underflow
// range); the leaf-pair sum is unscaled in double precision.  Weights are
// stored divided by the largest weight.
#include <cstring>  // rocprim uses memset without including it
#include <rocprim/rocprim.hpp>

#include <algorithm>

#include "gs_series.h"

namespace gs {

namespace {

constexpr int kW = 64;
constexpr int kWaves = 4;  // waves per run
constexpr int kHB = 8;     // bandwidths per block

__global__ void base_records_kernel(const double* __restrict__ xr, const double* __restrict__ wr,
                                    const int32_t* __restrict__ leaf_of_pos,
                                    const double* __restrict__ rctr, int64_t n, int D, int rs,
                                    const unsigned long long* __restrict__ wmax_bits,
                                    float* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* c = rctr + (int64_t)leaf_of_pos[i] * D;
  float* o = rec + i * rs;
  for (int d = 0; d < D; ++d) o[d] = (float)(xr[i * D + d] - c[d]);
  o[D] = (float)(wr[i] / __longlong_as_double((long long)*wmax_bits));
  for (int k = D + 1; k < rs; ++k) o[k] = 0.0f;
}

// One workgroup per base group {h, Q, first, n}: key (Q, h / 8, R), bit h % 8.
__global__ void fuse_keys_kernel(const int4* __restrict__ grp, int ng, const int32_t* __restrict__ ent,
                                 int rbits, int hbits, unsigned long long* __restrict__ key,
                                 uint8_t* __restrict__ bit) {
  const int gi = blockIdx.x;
  if (gi >= ng) return;
  const int4 g = grp[gi];
  const unsigned long long hb = (unsigned long long)(g.x / kHB);
  const unsigned long long hi = ((unsigned long long)g.y << (hbits + rbits)) | (hb << rbits);
  const uint8_t b = (uint8_t)(1u << (g.x % kHB));
  for (int e = threadIdx.x; e < g.w; e += blockDim.x) {
    key[g.z + e] = hi | (unsigned long long)(ent[g.z + e] >> 4);
    bit[g.z + e] = b;
  }
}

struct BitOr {
  __device__ __host__ uint8_t operator()(uint8_t a, uint8_t b) const { return (uint8_t)(a | b); }
};

// Run heads (first entry of each (Q, block)) and the number of point pairs
// whose squared distance the fused kernel forms.
__global__ void run_flags_kernel(const unsigned long long* __restrict__ ukey, int n, int rbits, int hbits,
                                 const int32_t* __restrict__ qcount, const int32_t* __restrict__ rcount,
                                 int32_t* __restrict__ flag, unsigned long long* __restrict__ dist_evals) {
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
  if ((threadIdx.x % kW) == 0 && pe) atomicAdd(dist_evals, pe);
}

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

// Sweep of one reference leaf for NA bandwidths: for every point r,
//   part[j] += w_r exp2(shiftc[j] - |u_q - u_r|^2 shc[j]),  j < NA.
// The record addresses are wave-uniform (scalar loads).
template <int DC, int NA>
__device__ __forceinline__ void sweep(const float* __restrict__ rp, int rn, int rs, int D,
                                      const float* uq, const float* shc, const float* shiftc,
                                      float* part) {
#pragma unroll 2
  for (int r = 0; r < rn; ++r) {
    const float* x = rp + r * rs;
    float d2 = 0.0f;
#pragma unroll
    for (int d = 0; d < DC; ++d) {
      if (d < D) {
        const float dd = uq[d] - x[d];
        d2 = fmaf(dd, dd, d2);
      }
    }
    const float wr = x[D];
#pragma unroll
    for (int j = 0; j < NA; ++j)
      part[j] = fmaf(wr, __builtin_amdgcn_exp2f(fmaf(-d2, shc[j], shiftc[j])), part[j]);
  }
}

template <int DT>
__global__ __launch_bounds__(kW* kWaves) void base_fused_kernel(
    const int32_t* __restrict__ run_start, int nruns, const unsigned long long* __restrict__ ukey,
    const uint8_t* __restrict__ umask, int rbits, int hbits, int hc0, int hc1, NodeView qt, NodeView rt,
    const double* __restrict__ xq_perm, const float* __restrict__ rec, int Drt, int rs_rt,
    const float* __restrict__ s2, const unsigned long long* __restrict__ wmax_bits, int Mq,
    double* __restrict__ gx) {
  __shared__ double red[kWaves - 1][kHB][kW];
  constexpr int DC = DT > 0 ? DT : kMaxD;
  const int D = DT > 0 ? DT : Drt;
  const int rs = DT > 0 ? (DT + 4) / 4 * 4 : rs_rt;
  // Consecutive runs (neighbouring query leaves, which share reference
  // leaves) go to the same XCD: workgroups are dealt to the 8 XCDs
  // round-robin, so block b takes run (b % 8) * per + b / 8.
  const int per = (nruns + 7) / 8;
  const int run = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (run >= nruns) return;
  const int e0 = run_start[run], e1 = run_start[run + 1];
  const unsigned long long k0 = ukey[e0];
  const int Q = (int)(k0 >> (hbits + rbits));
  const int h0 = (int)((k0 >> rbits) & ((1ull << hbits) - 1)) * kHB;
  const unsigned long long rmask = (1ull << rbits) - 1;
  const int qb = qt.begin[Q], qn = qt.count[Q];
  const int lane = threadIdx.x % kW;
  // wave index as a wave-uniform value, so the run's entries (and the
  // reference points they name) are read with scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kW);
  for (int base = 0; base < qn; base += kW) {
    const bool active = base + lane < qn;
    const int qpos = qb + base + (active ? lane : 0);
    double xq[DC];
#pragma unroll
    for (int d = 0; d < DC; ++d)
      if (d < D) xq[d] = xq_perm[(int64_t)qpos * D + d];
    double acc[kHB];
#pragma unroll
    for (int k = 0; k < kHB; ++k) acc[k] = 0.0;
    for (int e = e0 + wave; e < e1; e += kWaves) {
      const int R = (int)(ukey[e] & rmask);
      const unsigned m = umask[e];
      const double* cR = rt.ctr + (int64_t)R * D;
      const double* lR = rt.lo + (int64_t)R * D;
      const double* hR = rt.hi + (int64_t)R * D;
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
      // Compact the entry's bandwidths: j-th set bit of m -> shc[j] (uniform),
      // shiftc[j] = the lane's underflow shift for that bandwidth.
      const int na = __builtin_popcount(m);
      float shc[kHB], shiftc[kHB], part[kHB];
      {
        unsigned mm = m;
#pragma unroll
        for (int j = 0; j < kHB; ++j) {
          const int k = mm ? __builtin_ctz(mm) : 0;
          mm &= mm - 1;
          shc[j] = s2[h0 + k];
          shiftc[j] = (float)box2 * shc[j];
          part[j] = 0.0f;
        }
      }
      const float* rp = rec + (int64_t)rt.begin[R] * rs;
      const int rn = rt.count[R];
      switch (na) {
        case 1: sweep<DC, 1>(rp, rn, rs, D, uq, shc, shiftc, part); break;
        case 2: sweep<DC, 2>(rp, rn, rs, D, uq, shc, shiftc, part); break;
        case 3: sweep<DC, 3>(rp, rn, rs, D, uq, shc, shiftc, part); break;
        case 4: sweep<DC, 4>(rp, rn, rs, D, uq, shc, shiftc, part); break;
        case 5: sweep<DC, 5>(rp, rn, rs, D, uq, shc, shiftc, part); break;
        case 6: sweep<DC, 6>(rp, rn, rs, D, uq, shc, shiftc, part); break;
        case 7: sweep<DC, 7>(rp, rn, rs, D, uq, shc, shiftc, part); break;
        default: sweep<DC, 8>(rp, rn, rs, D, uq, shc, shiftc, part); break;
      }
      {
        unsigned mm = m;
#pragma unroll
        for (int j = 0; j < kHB; ++j) {
          if (mm == 0) break;
          const int k = __builtin_ctz(mm);
          mm &= mm - 1;
          const float fi = floorf(shiftc[j]);
          const double v = ldexp((double)(part[j] * __builtin_amdgcn_exp2f(fi - shiftc[j])), -(int)fi);
#pragma unroll
          for (int t = 0; t < kHB; ++t)
            if (t == k) acc[t] += v;
        }
      }
    }
    if (wave > 0) {
#pragma unroll
      for (int k = 0; k < kHB; ++k) red[wave - 1][k][lane] = acc[k];
    }
    __syncthreads();
    if (wave == 0 && active) {
      const double wscale = __longlong_as_double((long long)*wmax_bits);
#pragma unroll
      for (int k = 0; k < kHB; ++k) {
        double v = acc[k];
#pragma unroll
        for (int w = 0; w < kWaves - 1; ++w) v += red[w][k][lane];
        if (h0 + k >= hc0 && h0 + k < hc1) gx[(int64_t)(h0 + k) * Mq + qpos] = v * wscale;
      }
    }
    __syncthreads();
  }
}

int bits_for(int64_t n) {
  int b = 1;
  while ((1ll << b) < n) ++b;
  return b;
}

template <int DT>
void launch_fused_t(const BaseFusedArgs& a, const BaseFusedPlan& p, hipStream_t s) {
  const int nb = (p.nruns + 7) / 8 * 8;
  hipLaunchKernelGGL((base_fused_kernel<DT>), dim3((unsigned)nb), dim3(kW * kWaves), 0, s, a.run_start,
                     p.nruns, a.ukey, a.umask, p.rbits, p.hbits, a.hc0, a.hc1, a.qt, a.rt, a.xq_perm,
                     a.rec, a.D, base_record_stride(a.D), a.s2, a.wmax_bits, a.Mq, a.gx);
}

}  // namespace

int base_record_stride(int D) { return (D + 1 + 3) / 4 * 4; }

hipError_t launch_base_records(const double* xr_perm, const double* wr_perm, const int32_t* leaf_of_pos,
                               const double* rctr, int64_t n, int D, const unsigned long long* wmax_bits,
                               float* rec, hipStream_t s) {
  hipLaunchKernelGGL(base_records_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, xr_perm,
                     wr_perm, leaf_of_pos, rctr, n, D, base_record_stride(D), wmax_bits, rec);
  return hipGetLastError();
}

size_t base_fused_temp_bytes(int64_t n) {
  size_t b1 = 0, b2 = 0, b3 = 0;
  (void)rocprim::radix_sort_pairs((void*)nullptr, b1, (const unsigned long long*)nullptr,
                                  (unsigned long long*)nullptr, (const uint8_t*)nullptr,
                                  (uint8_t*)nullptr, (size_t)n, 0, 64);
  (void)rocprim::reduce_by_key((void*)nullptr, b2, (const unsigned long long*)nullptr,
                               (const uint8_t*)nullptr, (size_t)n, (unsigned long long*)nullptr,
                               (uint8_t*)nullptr, (int32_t*)nullptr, BitOr(),
                               rocprim::equal_to<unsigned long long>());
  (void)rocprim::exclusive_scan((void*)nullptr, b3, (const int32_t*)nullptr, (int32_t*)nullptr, 0,
                                (size_t)n, rocprim::plus<int32_t>());
  return std::max(b1, std::max(b2, b3));
}

hipError_t plan_base_fused(const BaseFusedArgs& a, BaseFusedPlan* p, hipStream_t s) {
  p->nruns = 0;
  const int64_t n = a.n_entries;
  if (n == 0 || a.n_groups == 0) return hipSuccess;
  p->rbits = bits_for(a.n_rnodes + 1);
  p->hbits = bits_for(a.n_hblocks + 1);
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
                             a.n_unique, BitOr(), rocprim::equal_to<unsigned long long>(), s);
  if (e != hipSuccess) return e;
  int32_t nu = 0;
  e = hipMemcpyAsync(&nu, a.n_unique, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (nu <= 0 || nu > n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(run_flags_kernel, dim3((unsigned)ceil_div(nu, 256)), dim3(256), 0, s, a.ukey, nu,
                     p->rbits, p->hbits, a.qt.count, a.rt.count, a.flag, a.dist_evals);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  bytes = a.temp_bytes;
  e = rocprim::exclusive_scan(a.temp, bytes, a.flag, a.pos, 0, (size_t)nu, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(run_scatter_kernel, dim3((unsigned)ceil_div(nu, 256)), dim3(256), 0, s, a.flag,
                     a.pos, nu, a.run_start, a.n_unique);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int32_t nr = 0;
  e = hipMemcpyAsync(&nr, a.n_unique, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if (nr <= 0 || nr > nu) return hipErrorInvalidValue;
  p->nruns = nr;
  return hipSuccess;
}

hipError_t launch_base_fused(const BaseFusedArgs& a, const BaseFusedPlan& p, hipStream_t s) {
  if (p.nruns == 0) return hipSuccess;
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
  return hipGetLastError();
}

}  // namespace gs
