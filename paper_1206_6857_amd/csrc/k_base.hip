// Exhaustive base cases of the dual-tree traversal (DITOBase, Figure 7):
// for every base pair (Q leaf, R leaf) of a bandwidth h,
//     gx[h][q] += sum_{r in R} w_r exp(-|x_q - x_r|^2 / 2h^2),   q in Q.
//
// One wave handles one run of base groups of a (h, Q) key, so it owns gx[h][q]
// for the points of Q and writes them once, deterministically.  Lanes hold the
// query points; each reference leaf is staged into LDS with coalesced loads and
// swept with broadcast reads.
//
// Precision: reference coordinates are stored relative to their leaf centre
// in float (u_r = x_r - c_R), and each lane forms u_q = x_q - c_R in double
// before rounding to float, so the float difference u_q - u_r is accurate to
// ~2^-24 of the pair's extent.  To keep far pairs out of the float underflow
// range, every term is scaled by exp(+d_box^2/2h^2), where d_box is the
// distance from x_q to R's bounding box (a lower bound of |x_q - x_r|, so each
// scaled term is <= 1); the per-pair sum is unscaled in double precision
// (exp2 of the fractional part in float, ldexp of the integer part).  Weights
// are stored divided by the largest weight.
#include "gs_series.h"

namespace gs {

namespace {

constexpr int kW = 64;

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

template <int DT>
__global__ __launch_bounds__(kW) void base_kernel(SortedGroups g, const int32_t* __restrict__ ent,
                                                  NodeView qt, NodeView rt,
                                                  const double* __restrict__ xq_perm,
                                                  const float* __restrict__ rec, int Drt, int rs,
                                                  const float* __restrict__ s2,
                                                  const unsigned long long* __restrict__ wmax_bits,
                                                  int Mq, double* __restrict__ gx) {
  extern __shared__ float srec[];  // [kW][rs]: the reference chunk being swept
  constexpr int DC = DT > 0 ? DT : kMaxD;
  const int D = DT > 0 ? DT : Drt;
  const int i = blockIdx.x;
  if (i >= g.n || (i > 0 && g.key[i] == g.key[i - 1])) return;
  const int4 g0 = g.grp[g.order[i]];
  const int h = g0.x, Q = g0.y;
  const float sh = s2[h];
  const double wscale = __longlong_as_double((long long)*wmax_bits);
  const int qb = qt.begin[Q], qn = qt.count[Q];
  const int lane = threadIdx.x;
  const int rs4 = rs / 4;
  for (int base = 0; base < qn; base += kW) {
    const bool active = base + lane < qn;
    const int qpos = qb + base + (active ? lane : 0);
    double xq[DC];
#pragma unroll
    for (int d = 0; d < DC; ++d)
      if (d < D) xq[d] = xq_perm[(int64_t)qpos * D + d];
    double acc = 0.0;
    for (int j = i; j < g.n && (j == i || g.key[j] == g.key[j - 1]); ++j) {
      const int4 gr = g.grp[g.order[j]];
      for (int e = gr.z; e < gr.z + gr.w; ++e) {
        const int R = ent[e] >> 4;
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
        const float shift = (float)box2 * sh;
        const int rb = rt.begin[R], rn = rt.count[R];
        float part = 0.0f;
        for (int c0 = 0; c0 < rn; c0 += kW) {
          const int cn = rn - c0 < kW ? rn - c0 : kW;
          __syncthreads();
          {
            const float4* src = reinterpret_cast<const float4*>(rec + (int64_t)(rb + c0) * rs);
            float4* dst = reinterpret_cast<float4*>(srec);
            for (int t = lane; t < cn * rs4; t += kW) dst[t] = src[t];
          }
          __syncthreads();
#pragma unroll 4
          for (int r = 0; r < cn; ++r) {
            const float* x = srec + r * rs;
            float d2 = 0.0f;
#pragma unroll
            for (int d = 0; d < DC; ++d) {
              if (d < D) {
                const float dd = uq[d] - x[d];
                d2 = fmaf(dd, dd, d2);
              }
            }
            part = fmaf(x[D], __builtin_amdgcn_exp2f(fmaf(-d2, sh, shift)), part);
          }
        }
        const float fi = floorf(shift);
        acc += ldexp((double)(part * __builtin_amdgcn_exp2f(fi - shift)), -(int)fi);
      }
    }
    if (active) gx[(int64_t)h * Mq + qpos] = acc * wscale;
  }
}

template <int DT>
void launch_base_t(const SortedGroups& g, const int32_t* ent, const NodeView& qt, const NodeView& rt,
                   const double* xq_perm, const float* rec, int D, const float* s2,
                   const unsigned long long* wb, int Mq, double* gx, hipStream_t s) {
  const int rs = base_record_stride(D);
  hipLaunchKernelGGL((base_kernel<DT>), dim3(g.n), dim3(kW), (size_t)kW * rs * sizeof(float), s, g,
                     ent, qt, rt, xq_perm, rec, D, rs, s2, wb, Mq, gx);
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

hipError_t launch_base(const SortedGroups& g, const int32_t* ent, const NodeView& qt,
                       const NodeView& rt, const double* xq_perm, const float* rec, int D,
                       const float* s2, const unsigned long long* wb, int Mq, double* gx,
                       hipStream_t s) {
  if (g.n == 0) return hipSuccess;
  switch (D) {
    case 1: launch_base_t<1>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
    case 2: launch_base_t<2>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
    case 3: launch_base_t<3>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
    case 4: launch_base_t<4>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
    case 5: launch_base_t<5>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
    case 8: launch_base_t<8>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
    case 16: launch_base_t<16>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
    default: launch_base_t<0>(g, ent, qt, rt, xq_perm, rec, D, s2, wb, Mq, gx, s); break;
  }
  return hipGetLastError();
}

}  // namespace gs
