// Least-squares cross-validation score of a Gaussian kernel density estimate
// (the bandwidth-selection criterion of the experiments, section 7):
//
//   LSCV(h) = (4 pi h^2)^(-D/2) / N^2 * sum_i G_{sqrt2 h}(x_i)
//             - 2 (2 pi h^2)^(-D/2) / (N (N-1)) * sum_i (G_h(x_i) - 1),
//
// where G_h(x_i) = sum_j exp(-|x_i - x_j|^2 / 2h^2) over the points themselves
// (the first term is the integral of the squared estimate, a double sum
// because two Gaussians of variance h^2 convolve to one of variance 2h^2; the
// second is the leave-one-out estimate at every point).  Given the per-point
// sums with relative error eps each (Theorem 2), the score is off by at most
//   eps/(1-eps) * ((4 pi h^2)^(-D/2)/N^2 * S2~ + 2 (2 pi h^2)^(-D/2)/(N(N-1)) * S1~)
// with S2~ = sum_i G~_{sqrt2 h}(x_i) and S1~ = sum_i G~_h(x_i).
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kT = 256;

// One workgroup per row of G[rows][N]: the row sum in a fixed order.
__global__ __launch_bounds__(kT) void row_sums_kernel(const double* __restrict__ G, int64_t N,
                                                      double* __restrict__ sums) {
  __shared__ double part[kT];
  const int row = blockIdx.x;
  const double* g = G + (int64_t)row * N;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += kT) s += g[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[row] = part[0];
}

// sums[0..n_h) = S1~ (bandwidths h), sums[n_h..2 n_h) = S2~ (sqrt(2) h).
__global__ void lscv_combine_kernel(const double* __restrict__ sums, const double* __restrict__ hs, int n_h,
                                    int64_t N, int D, double eps, double* __restrict__ score,
                                    double* __restrict__ bound) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_h) return;
  const double h = hs[k];
  const double pi = 3.14159265358979323846;
  const double n = (double)N;
  const double a = pow(4.0 * pi * h * h, -0.5 * D) / (n * n);
  const double b = 2.0 * pow(2.0 * pi * h * h, -0.5 * D) / (n * (n - 1.0));
  const double s1 = sums[k], s2 = sums[n_h + k];
  score[k] = a * s2 - b * (s1 - n);
  if (bound) bound[k] = eps / (1.0 - eps) * (a * s2 + b * s1);
}

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_lscv_reduce(const double* G, int rows, int64_t N, double* sums, hipStream_t s) {
  hipLaunchKernelGGL(row_sums_kernel, dim3((unsigned)rows), dim3(kT), 0, s, G, N, sums);
  return hipGetLastError();
}

hipError_t launch_lscv_combine(const double* sums, const double* hs, int n_h, int64_t N, int D, double eps,
                               double* score, double* bound, hipStream_t s) {
  hipLaunchKernelGGL(lscv_combine_kernel, dim3((unsigned)ceil_div(n_h, 64)), dim3(64), 0, s, sums, hs, n_h, N,
                     D, eps, score, bound);
  return hipGetLastError();
}

}  // namespace gs
