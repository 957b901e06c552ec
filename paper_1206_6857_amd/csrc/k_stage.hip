// Input staging: validation and layout conversion of caller arrays.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

// Copy row-major points into a structure-of-arrays copy x_soa[d][n] and a
// row-major copy x_aos[n][D].  Adding +0.0 turns -0.0 into +0.0, so that
// both zeros compare and sort as one value.  Any NaN or infinity raises
// *bad_flag.
__global__ void stage_points_kernel(const double* __restrict__ x, int64_t n, int D,
                                    double* __restrict__ x_soa, double* __restrict__ x_aos,
                                    int* __restrict__ bad_flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool bad = false;
  for (int d = 0; d < D; ++d) {
    double v = x[i * D + d] + 0.0;
    if (!isfinite(v)) bad = true;
    x_soa[(int64_t)d * n + i] = v;
    x_aos[i * D + d] = v;
  }
  if (bad) atomicOr(bad_flag, 1);
}

__global__ void check_positive_kernel(const double* __restrict__ v, int64_t n,
                                      int* __restrict__ bad_flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = v[i];
  if (!(a > 0.0) || !isfinite(a)) atomicOr(bad_flag, 2);
}

__global__ void check_finite_kernel(const double* __restrict__ v, int64_t n,
                                    int* __restrict__ bad_flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!isfinite(v[i])) atomicOr(bad_flag, 1);
}

hipError_t launch_stage_points(const double* x, int64_t n, int D, double* x_soa, double* x_aos,
                               int* bad_flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(stage_points_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, x, n,
                     D, x_soa, x_aos, bad_flag);
  return hipGetLastError();
}

hipError_t launch_check_positive(const double* v, int64_t n, int* bad_flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_positive_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, v,
                     n, bad_flag);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* v, int64_t n, int* bad_flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, v, n,
                     bad_flag);
  return hipGetLastError();
}

}  // namespace gs

namespace gs {

namespace {

__global__ void gather_rows_kernel(const double* __restrict__ src, const int32_t* __restrict__ perm,
                                   int64_t n, int D, double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * D) return;
  const int64_t i = t / D;
  const int d = (int)(t - i * D);
  dst[t] = src[(int64_t)perm[i] * D + d];
}

__global__ void gather_kernel(const double* __restrict__ src, const int32_t* __restrict__ perm,
                              int64_t n, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

__global__ void clear_bits_kernel(unsigned long long* __restrict__ out_bits) { *out_bits = 0ull; }

// Largest of positive doubles (their bit patterns order the same way): each
// thread a strided share, a block maximum, then one atomic per block.
__global__ __launch_bounds__(1024) void max_bits_kernel(const double* __restrict__ w, int64_t n,
                                                        unsigned long long* __restrict__ out_bits) {
  __shared__ unsigned long long part[16];
  unsigned long long v = 0ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(w[i]);
    v = b > v ? b : v;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < (int)(blockDim.x / 64); ++k) v = part[k] > v ? part[k] : v;
    if (v) atomicMax(out_bits, v);
  }
}

}  // namespace

hipError_t launch_gather_rows(const double* src, const int32_t* perm, int64_t n, int D, double* dst,
                              hipStream_t s) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)ceil_div(n * D, 256)), dim3(256), 0, s, src,
                     perm, n, D, dst);
  return hipGetLastError();
}

hipError_t launch_gather(const double* src, const int32_t* perm, int64_t n, double* dst,
                         hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, src, perm, n,
                     dst);
  return hipGetLastError();
}

hipError_t launch_max_positive(const double* w, int64_t n, unsigned long long* out_bits,
                               hipStream_t s) {
  hipLaunchKernelGGL(clear_bits_kernel, dim3(1), dim3(1), 0, s, out_bits);
  const int64_t blocks = std::min<int64_t>(ceil_div(n, 1024), 256);
  hipLaunchKernelGGL(max_bits_kernel, dim3((unsigned)blocks), dim3(1024), 0, s, w, n, out_bits);
  return hipGetLastError();
}

}  // namespace gs
