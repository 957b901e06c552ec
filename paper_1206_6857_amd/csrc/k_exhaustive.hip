// Plain exhaustive Gaussian summation over all query/reference pairs
// (the "Naive" algorithm of section 7), fused over a block of bandwidths.
//
// Each thread owns one query; reference records are staged through LDS in
// chunks and read as wave-uniform broadcasts.  Coordinates are carried as a
// float pair (hi, lo) with x = hi + lo to ~2^-48, so the difference
// x_q - x_r is accurate to ~2^-24 relative even for points much closer
// together than their magnitude.  The squared distance is computed once per
// point pair and reused for every bandwidth of the block:
//     K = exp2(-d^2 * log2(e) / (2 h^2))   (one v_exp_f32)
// Weights are stored divided by the largest weight, so every float term is
// at most 1.  Per-chunk partial sums are kept in float (at most 256 positive
// terms) and folded into a double accumulator after every chunk.
//
// Underflow: a query far from every reference (relative to h) has all its
// float terms below the normal range.  When a sum ends below 2^-90, the whole
// workgroup reruns its reference range once more for that bandwidth block with
// every exponent shifted by the query's own smallest d^2 (found in an extra
// distance-only pass), and scales the result back in double precision.  The
// rerun happens only for such isolated queries.
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kThreads = 256;

struct HBlock {
  float s[kMaxHBlock];  // log2(e) / (2 h^2) per bandwidth of the block
};

__global__ void exhaustive_records_kernel(const double* __restrict__ x, const double* __restrict__ w,
                                          const unsigned long long* __restrict__ wmax_bits,
                                          int64_t n, int D, int rs, float* __restrict__ rec) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float* o = rec + i * rs;
  for (int d = 0; d < D; ++d) {
    double v = x[i * D + d];
    float hi = (float)v;
    o[d] = hi;
    o[D + d] = (float)(v - (double)hi);
  }
  o[2 * D] = (float)(w[i] / __longlong_as_double((long long)*wmax_bits));
  for (int k = 2 * D + 1; k < rs; ++k) o[k] = 0.0f;
}

template <int DT, int HB>
__global__ __launch_bounds__(kThreads) void exhaustive_kernel(
    const double* __restrict__ xq, int64_t M, const float* __restrict__ rec, int64_t N, int Drt,
    int rs, int chunk, int64_t r_per_split, HBlock hb, int h0, int n_h,
    const unsigned long long* __restrict__ wmax_bits, double* __restrict__ partial) {
  extern __shared__ float lds[];
  constexpr int DC = DT > 0 ? DT : kMaxD;
  const int D = DT > 0 ? DT : Drt;
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int split = blockIdx.y;
  const int64_t rb = (int64_t)split * r_per_split;
  const int64_t re = rb + r_per_split < N ? rb + r_per_split : N;

  float qh[DC], ql[DC];
  const int64_t qc = q < M ? q : M - 1;
#pragma unroll
  for (int d = 0; d < DC; ++d) {
    if (d < D) {
      double v = xq[qc * D + d];
      qh[d] = (float)v;
      ql[d] = (float)(v - (double)qh[d]);
    }
  }
  auto dist2 = [&](const float* r) {
    float d2 = 0.0f;
#pragma unroll
    for (int d = 0; d < DC; ++d) {
      if (d < D) {
        float dd = (qh[d] - r[d]) + (ql[d] - r[D + d]);
        d2 = fmaf(dd, dd, d2);
      }
    }
    return d2;
  };
  auto stage = [&](int64_t c, int cn) {
    __syncthreads();
    const float4* src = reinterpret_cast<const float4*>(rec + c * rs);
    float4* dst = reinterpret_cast<float4*>(lds);
    const int n4 = cn * rs / 4;
    for (int t = threadIdx.x; t < n4; t += kThreads) dst[t] = src[t];
    __syncthreads();
  };

  // Main pass: float terms exp2(-d2 * s_k) <= 1.
  double acc[HB];
  float part[HB];
#pragma unroll
  for (int k = 0; k < HB; ++k) {
    acc[k] = 0.0;
    part[k] = 0.0f;
  }
  for (int64_t c = rb; c < re; c += chunk) {
    const int cn = (int)(re - c < chunk ? re - c : chunk);
    stage(c, cn);
    for (int j = 0; j < cn; ++j) {
      const float* r = lds + j * rs;
      const float d2 = dist2(r);
      const float wr = r[2 * D];
#pragma unroll
      for (int k = 0; k < HB; ++k)
        part[k] = fmaf(wr, __builtin_amdgcn_exp2f(-d2 * hb.s[k]), part[k]);
    }
#pragma unroll
    for (int k = 0; k < HB; ++k) {
      acc[k] += (double)part[k];
      part[k] = 0.0f;
    }
  }

  // Rescue pass for sums that fell below 2^-90 (see the file comment).
  int need = 0;
#pragma unroll
  for (int k = 0; k < HB; ++k) need |= acc[k] < 0x1p-90;
  if (q >= M) need = 0;
  if (__syncthreads_or(need)) {
    float m2 = INFINITY;
    for (int64_t c = rb; c < re; c += chunk) {
      const int cn = (int)(re - c < chunk ? re - c : chunk);
      stage(c, cn);
      for (int j = 0; j < cn; ++j) m2 = fminf(m2, dist2(lds + j * rs));
    }
    float shift[HB];
#pragma unroll
    for (int k = 0; k < HB; ++k) shift[k] = m2 * hb.s[k];
    double accs[HB];
#pragma unroll
    for (int k = 0; k < HB; ++k) accs[k] = 0.0;
    for (int64_t c = rb; c < re; c += chunk) {
      const int cn = (int)(re - c < chunk ? re - c : chunk);
      stage(c, cn);
      for (int j = 0; j < cn; ++j) {
        const float* r = lds + j * rs;
        const float d2 = dist2(r);
        const float wr = r[2 * D];
#pragma unroll
        for (int k = 0; k < HB; ++k)
          part[k] = fmaf(wr, __builtin_amdgcn_exp2f(fmaf(-d2, hb.s[k], shift[k])), part[k]);
      }
#pragma unroll
      for (int k = 0; k < HB; ++k) {
        accs[k] += (double)part[k];
        part[k] = 0.0f;
      }
    }
#pragma unroll
    for (int k = 0; k < HB; ++k)
      if (acc[k] < 0x1p-90) acc[k] = accs[k] * exp2(-(double)shift[k]);
  }
  const double w_scale = __longlong_as_double((long long)*wmax_bits);
  if (q < M) {
#pragma unroll
    for (int k = 0; k < HB; ++k)
      partial[((int64_t)split * n_h + h0 + k) * M + q] = acc[k] * w_scale;
  }
}

__global__ void exhaustive_reduce_kernel(const double* __restrict__ partial, int n_split,
                                         int64_t total, double* __restrict__ G) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double s = 0.0;
  for (int k = 0; k < n_split; ++k) s += partial[(int64_t)k * total + i];
  G[i] = s;
}

int chunk_for(int rs) {
  int c = 8192 / rs;
  if (c > 256) c = 256;
  if (c < 16) c = 16;
  return c;
}

int splits_for(int64_t M, int64_t N, int chunk) {
  int64_t qb = ceil_div(M, kThreads);
  int64_t s = ceil_div(2048, qb);
  int64_t maxs = ceil_div(N, chunk);
  if (s > maxs) s = maxs;
  if (s < 1) s = 1;
  if (s > 4096) s = 4096;
  return (int)s;
}

template <int DT, int HB>
void launch_one(dim3 grid, size_t lds, hipStream_t st, const double* xq, int64_t M,
                const float* rec, int64_t N, int D, int rs, int chunk, int64_t rps,
                const HBlock& hb, int h0, int n_h, const unsigned long long* wb, double* partial) {
  hipLaunchKernelGGL((exhaustive_kernel<DT, HB>), grid, dim3(kThreads), lds, st, xq, M, rec, N, D,
                     rs, chunk, rps, hb, h0, n_h, wb, partial);
}

template <int DT>
void launch_hb(int hbn, dim3 grid, size_t lds, hipStream_t st, const double* xq, int64_t M,
               const float* rec, int64_t N, int D, int rs, int chunk, int64_t rps,
               const HBlock& hb, int h0, int n_h, const unsigned long long* wb, double* partial) {
  switch (hbn) {
    case 16: launch_one<DT, 16>(grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
    case 8: launch_one<DT, 8>(grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
    case 4: launch_one<DT, 4>(grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
    case 2: launch_one<DT, 2>(grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
    default: launch_one<DT, 1>(grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
  }
}

}  // namespace

int exhaustive_record_stride(int D) { return ((2 * D + 1) + 3) / 4 * 4; }

hipError_t launch_exhaustive_records(const double* x_aos, const double* w, int64_t n, int D,
                                     float* rec, unsigned long long* wmax_bits, hipStream_t s) {
  hipError_t e = launch_max_positive(w, n, wmax_bits, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(exhaustive_records_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                     x_aos, w, wmax_bits, n, D, exhaustive_record_stride(D), rec);
  return hipGetLastError();
}

size_t exhaustive_partial_elems(int64_t M, int64_t N, int n_h) {
  // the chunk depends on D; the smallest chunk gives a safe upper bound
  return (size_t)splits_for(M, N, 16) * (size_t)n_h * (size_t)M;
}

size_t exhaustive_partial_elems_exact(int64_t M, int64_t N, int D, int n_h) {
  const int chunk = chunk_for(exhaustive_record_stride(D));
  const int n_split = splits_for(M, N, chunk);
  const int64_t rps = ceil_div(ceil_div(N, n_split), chunk) * chunk;
  return (size_t)ceil_div(N, rps) * (size_t)n_h * (size_t)M;
}

hipError_t launch_exhaustive(const double* xq, int64_t M, const float* rec, int64_t N, int D,
                             const double* hs, int n_h, const unsigned long long* wb,
                             double* partial, double* G, hipStream_t st) {
  const int rs = exhaustive_record_stride(D);
  const int chunk = chunk_for(rs);
  const int n_split = splits_for(M, N, chunk);
  const int64_t rps = ceil_div(ceil_div(N, n_split), chunk) * chunk;
  const int n_split_eff = (int)ceil_div(N, rps);
  dim3 grid((unsigned)ceil_div(M, kThreads), (unsigned)n_split_eff);
  const size_t lds = (size_t)chunk * rs * sizeof(float);
  int h0 = 0;
  while (h0 < n_h) {
    int rem = n_h - h0;
    int hbn = rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
    HBlock hb;
    for (int k = 0; k < kMaxHBlock; ++k) {
      double h = hs[h0 + (k < hbn ? k : 0)];
      hb.s[k] = (float)(1.4426950408889634 / (2.0 * h * h));
    }
    switch (D) {
      case 1: launch_hb<1>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
      case 2: launch_hb<2>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
      case 3: launch_hb<3>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
      case 4: launch_hb<4>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
      case 5: launch_hb<5>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
      case 8: launch_hb<8>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
      case 16: launch_hb<16>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
      default: launch_hb<0>(hbn, grid, lds, st, xq, M, rec, N, D, rs, chunk, rps, hb, h0, n_h, wb, partial); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    h0 += hbn;
  }
  int64_t total = (int64_t)n_h * M;
  hipLaunchKernelGGL(exhaustive_reduce_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0,
                     st, partial, n_split_eff, total, G);
  return hipGetLastError();
}

}  // namespace gs
