// Learned pair policy: features of a node pair, the cost-predicting network
// (inference on MFMA in half precision), and its training (gradient and Adam,
// single precision).
//
// The paper decides among its approximations with an operation-count rule
// (section 6, Figure 6) and remarks that the cut-offs are rough.  The policy
// predicts, from the pair's geometry only, the log2 cost of each action (DH,
// DL, H2L, recurse); the traversal takes the cheapest predicted action, and a
// series method is taken only if its error bound admits it (Lemmas 4-6, the
// same test as the rule), so Theorem 2 holds whatever the network predicts.
//
// Network: x[16] standardised -> 64 ReLU -> 64 ReLU -> 4.  Parameters, float:
// W1[64][16], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].
//
// Inference computes the transposed products, 16 pairs per wave and step:
//   H1^T = relu(W1 X^T + b1), H2^T = relu(W2 H1^T + b2), Y^T = W3 H2^T + b3,
// with v_mfma_f32_16x16x16_f16.  In the transposed form the accumulator layout
// of one 16-row block (lane = column + 16 * (row / 4), element row % 4) is the
// B-operand layout of the next product's 16-deep k-step, so the hidden
// activations never leave registers.  The weights are packed on the host in
// the A-operand layout (lane = row + 16 * (k / 4), element k % 4).
#include "gs_policy.h"

namespace gs {

namespace {

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kW = 64;

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

// Features k0..k0+3 of pair (h, Q, R) (k0 a multiple of 4):
//   0 log2 N_Q, 1 log2 N_R, 2 log2(1 + dmin/h), 3 log2(1 + dmax/h), 4 log2 h,
//   5 log2(1 + rinf_Q/h), 6 log2(1 + rinf_R/h), 7 [Q leaf], 8 [R leaf],
//   9 D/16, 10..15 zero.
__device__ void pair_features4(const PolicyTreeView& qt, const PolicyTreeView& rt, int D, int Q, int R,
                               double h, double ih, int k0, float* f) {
  f[0] = f[1] = f[2] = f[3] = 0.0f;
  if (k0 == 0) {
    double dmin2, dmax2;
    box_dist2(qt.lo + (int64_t)Q * D, qt.hi + (int64_t)Q * D, rt.lo + (int64_t)R * D,
              rt.hi + (int64_t)R * D, D, &dmin2, &dmax2);
    f[0] = (float)log2((double)qt.count[Q]);
    f[1] = (float)log2((double)rt.count[R]);
    f[2] = (float)log2(1.0 + sqrt(dmin2) * ih);
    f[3] = (float)log2(1.0 + sqrt(dmax2) * ih);
  } else if (k0 == 4) {
    f[0] = (float)log2(h);
    f[1] = (float)log2(1.0 + qt.rinf[Q] * ih);
    f[2] = (float)log2(1.0 + rt.rinf[R] * ih);
    f[3] = qt.left[Q] < 0 ? 1.0f : 0.0f;
  } else if (k0 == 8) {
    f[0] = rt.left[R] < 0 ? 1.0f : 0.0f;
    f[1] = (float)D / 16.0f;
  }
}

// Raw features of every pair of a frontier level, [pair][16].
__global__ void policy_features_kernel(int npair, PolicyPairs pp, PolicyTreeView qt, PolicyTreeView rt,
                                       int D, float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)npair * 4) return;
  const int g = (int)(i / 4), k0 = (int)(i % 4) * 4;
  const int s = pp.seg[g];
  const int h = pp.h[s];
  float f[4];
  pair_features4(qt, rt, D, pp.Q[s], pp.R[g], pp.hs[h], pp.invh[h], k0, f);
  for (int e = 0; e < 4; ++e) feat[(int64_t)g * 16 + k0 + e] = f[e];
}

__device__ __forceinline__ floatx4 mfma16(half4 a, half4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ half4 relu_half(floatx4 v) {
  half4 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) r[e] = (_Float16)(v[e] > 0.0f ? v[e] : 0.0f);
  return r;
}

// Scores of n pairs: from a frontier level (FROM_PAIRS) or from raw features.
// One wave per 16 pairs per step, grid-stride over the tiles.
template <bool FROM_PAIRS>
__global__ __launch_bounds__(kW) void policy_infer_kernel(int n, PolicyPairs pp, PolicyTreeView qt,
                                                          PolicyTreeView rt, int D,
                                                          const float* __restrict__ feat_in,
                                                          PolicyDevModel m, float4* __restrict__ scores) {
  const int lane = threadIdx.x;
  const int col = lane % 16, grp = lane / 16;
  // weights in A layout, biases in accumulator layout
  half4 w1[4], w2[4][4], w3[4];
  floatx4 b1[4], b2[4], b3;
  const half4* W = reinterpret_cast<const half4*>(m.wpack);
#pragma unroll
  for (int r = 0; r < 4; ++r) w1[r] = W[r * kW + lane];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int t = 0; t < 4; ++t) w2[r][t] = W[(4 + r * 4 + t) * kW + lane];
#pragma unroll
  for (int t = 0; t < 4; ++t) w3[t] = W[(20 + t) * kW + lane];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      b1[r][e] = m.b1[16 * r + 4 * grp + e];
      b2[r][e] = m.b2[16 * r + 4 * grp + e];
    }
    b3[e] = grp == 0 ? m.b3[e] : 0.0f;
  }
  float mu[4], isd[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    mu[e] = m.mu_x[4 * grp + e];
    isd[e] = m.isd_x[4 * grp + e];
  }
  const int ntiles = (n + 15) / 16;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int g = tile * 16 + col;
    float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (g < n) {
      if constexpr (FROM_PAIRS) {
        const int s = pp.seg[g];
        const int h = pp.h[s];
        pair_features4(qt, rt, D, pp.Q[s], pp.R[g], pp.hs[h], pp.invh[h], 4 * grp, f);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) f[e] = feat_in[(int64_t)g * 16 + 4 * grp + e];
      }
    }
    half4 xb;
#pragma unroll
    for (int e = 0; e < 4; ++e) xb[e] = (_Float16)(g < n ? (f[e] - mu[e]) * isd[e] : 0.0f);
    half4 h1[4], h2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) h1[r] = relu_half(mfma16(w1[r], xb, b1[r]));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      floatx4 acc = b2[r];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc = mfma16(w2[r][t], h1[t], acc);
      h2[r] = relu_half(acc);
    }
    floatx4 y = b3;
#pragma unroll
    for (int t = 0; t < 4; ++t) y = mfma16(w3[t], h2[t], y);
    if (grp == 0 && g < n) scores[g] = make_float4(y[0], y[1], y[2], y[3]);
  }
}

// Gradient of the masked squared loss, one wave per slice of the batch, lane j
// = hidden unit j.  Writes the wave's unnormalised sums: d/dtheta of
// sum m (y - t)^2 in the parameter order, then (sum m (y - t)^2, sum m).
__global__ __launch_bounds__(kW) void policy_grad_kernel(const float* __restrict__ rec,
                                                         const int32_t* __restrict__ idx, int n,
                                                         int per_wave, const float* __restrict__ theta,
                                                         PolicyNorm nm, float* __restrict__ partial) {
  __shared__ float W2s[kPolicyHidden][kPolicyHidden];
  __shared__ float h1s[kPolicyHidden], dh2s[kPolicyHidden];
  const int j = threadIdx.x;
  const float* W1 = theta;
  const float* b1 = W1 + kPolicyHidden * kPolicyIn;
  const float* W2 = b1 + kPolicyHidden;
  const float* b2 = W2 + kPolicyHidden * kPolicyHidden;
  const float* W3 = b2 + kPolicyHidden;
  const float* b3 = W3 + kPolicyOut * kPolicyHidden;
  float w1[kPolicyIn], w2[kPolicyHidden], w3[kPolicyOut];
  float gw1[kPolicyIn], gw2[kPolicyHidden], gw3[kPolicyOut], gb3[kPolicyOut];
  for (int k = 0; k < kPolicyIn; ++k) {
    w1[k] = W1[j * kPolicyIn + k];
    gw1[k] = 0.0f;
  }
  for (int i = 0; i < kPolicyHidden; ++i) {
    w2[i] = W2[j * kPolicyHidden + i];
    gw2[i] = 0.0f;
    W2s[i][j] = W2[i * kPolicyHidden + j];
  }
  for (int k = 0; k < kPolicyOut; ++k) {
    w3[k] = W3[k * kPolicyHidden + j];
    gw3[k] = 0.0f;
    gb3[k] = 0.0f;
  }
  const float bb1 = b1[j], bb2 = b2[j];
  float gb1 = 0.0f, gb2 = 0.0f, lsum = 0.0f, msum = 0.0f;
  __syncthreads();
  const int s0 = blockIdx.x * per_wave;
  const int s1 = min(n, s0 + per_wave);
  for (int s = s0; s < s1; ++s) {
    const float* r = rec + (int64_t)idx[s] * kPolicyRecord;
    float x[kPolicyIn];
    for (int k = 0; k < kPolicyIn; ++k) x[k] = (r[k] - nm.mu_x[k]) * nm.isd_x[k];
    float a1 = bb1;
    for (int k = 0; k < kPolicyIn; ++k) a1 = fmaf(w1[k], x[k], a1);
    const float hh1 = a1 > 0.0f ? a1 : 0.0f;
    h1s[j] = hh1;
    __syncthreads();
    float a2 = bb2;
    for (int i = 0; i < kPolicyHidden; ++i) a2 = fmaf(w2[i], h1s[i], a2);
    const float hh2 = a2 > 0.0f ? a2 : 0.0f;
    float dy[kPolicyOut];
    for (int k = 0; k < kPolicyOut; ++k) {
      float y = w3[k] * hh2;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) y += __shfl_xor(y, off, kW);
      y += b3[k];
      const float m = r[kPolicyIn + kPolicyOut + k];
      const float t = (r[kPolicyIn + k] - nm.mu_y) * nm.isd_y;
      const float e = m != 0.0f ? y - t : 0.0f;
      dy[k] = 2.0f * m * e;
      lsum = fmaf(m * e, e, lsum);
      msum += m;
    }
    float dh2 = 0.0f;
    for (int k = 0; k < kPolicyOut; ++k) {
      gw3[k] = fmaf(dy[k], hh2, gw3[k]);
      gb3[k] += dy[k];
      dh2 = fmaf(w3[k], dy[k], dh2);
    }
    dh2 = a2 > 0.0f ? dh2 : 0.0f;
    for (int i = 0; i < kPolicyHidden; ++i) gw2[i] = fmaf(dh2, h1s[i], gw2[i]);
    gb2 += dh2;
    dh2s[j] = dh2;
    __syncthreads();
    float dh1 = 0.0f;
    for (int i = 0; i < kPolicyHidden; ++i) dh1 = fmaf(W2s[i][j], dh2s[i], dh1);
    dh1 = a1 > 0.0f ? dh1 : 0.0f;
    for (int k = 0; k < kPolicyIn; ++k) gw1[k] = fmaf(dh1, x[k], gw1[k]);
    gb1 += dh1;
    __syncthreads();
  }
  float* out = partial + (int64_t)blockIdx.x * (kPolicyParams + 2);
  float* oW1 = out;
  float* ob1 = oW1 + kPolicyHidden * kPolicyIn;
  float* oW2 = ob1 + kPolicyHidden;
  float* ob2 = oW2 + kPolicyHidden * kPolicyHidden;
  float* oW3 = ob2 + kPolicyHidden;
  float* ob3 = oW3 + kPolicyOut * kPolicyHidden;
  for (int k = 0; k < kPolicyIn; ++k) oW1[j * kPolicyIn + k] = gw1[k];
  ob1[j] = gb1;
  for (int i = 0; i < kPolicyHidden; ++i) oW2[j * kPolicyHidden + i] = gw2[i];
  ob2[j] = gb2;
  for (int k = 0; k < kPolicyOut; ++k) oW3[k * kPolicyHidden + j] = gw3[k];
  if (j == 0) {
    for (int k = 0; k < kPolicyOut; ++k) ob3[k] = gb3[k];
    out[kPolicyParams] = lsum;
    out[kPolicyParams + 1] = msum;
  }
}

// Sum of the wave partials in wave order, divided by max(1, sum of masks);
// optionally one Adam step on theta.  stats[0] = loss, stats[1] = mask sum.
__global__ void policy_reduce_kernel(const float* __restrict__ partial, int nwaves, float* __restrict__ grad,
                                     float* __restrict__ theta, float* __restrict__ am,
                                     float* __restrict__ av, PolicyAdam ad, float* __restrict__ stats) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kPolicyParams) return;
  const int stride = kPolicyParams + 2;
  float msum = 0.0f;
  for (int w = 0; w < nwaves; ++w) msum += partial[(int64_t)w * stride + kPolicyParams + 1];
  const float inv = 1.0f / (msum > 1.0f ? msum : 1.0f);
  if (p == kPolicyParams) {
    float l = 0.0f;
    for (int w = 0; w < nwaves; ++w) l += partial[(int64_t)w * stride + kPolicyParams];
    stats[0] = l * inv;
    stats[1] = msum;
    return;
  }
  float g = 0.0f;
  for (int w = 0; w < nwaves; ++w) g += partial[(int64_t)w * stride + p];
  g *= inv;
  if (grad) grad[p] = g;
  if (theta) {
    const float m = ad.beta1 * am[p] + (1.0f - ad.beta1) * g;
    const float v = ad.beta2 * av[p] + (1.0f - ad.beta2) * g * g;
    am[p] = m;
    av[p] = v;
    const float mh = m / ad.bc1;
    const float vh = v / ad.bc2;
    theta[p] -= ad.lr * mh / (sqrtf(vh) + ad.eps);
  }
}

}  // namespace

hipError_t launch_policy_features(int npair, const PolicyPairs& pp, const PolicyTreeView& qt,
                                  const PolicyTreeView& rt, int D, float* feat, hipStream_t s) {
  if (npair == 0) return hipSuccess;
  hipLaunchKernelGGL(policy_features_kernel, dim3((unsigned)ceil_div((int64_t)npair * 4, 256)), dim3(256),
                     0, s, npair, pp, qt, rt, D, feat);
  return hipGetLastError();
}

static unsigned infer_grid(int n) {
  const int64_t tiles = ceil_div(n, 16);
  return (unsigned)std::min<int64_t>(tiles, 256 * 16);
}

hipError_t launch_policy_infer_pairs(int npair, const PolicyPairs& pp, const PolicyTreeView& qt,
                                     const PolicyTreeView& rt, int D, const PolicyDevModel& m,
                                     float4* scores, hipStream_t s) {
  if (npair == 0) return hipSuccess;
  hipLaunchKernelGGL(policy_infer_kernel<true>, dim3(infer_grid(npair)), dim3(kW), 0, s, npair, pp, qt, rt,
                     D, (const float*)nullptr, m, scores);
  return hipGetLastError();
}

hipError_t launch_policy_infer_features(int n, const float* feat, const PolicyDevModel& m, float4* scores,
                                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  PolicyPairs pp{};
  PolicyTreeView tv{};
  hipLaunchKernelGGL(policy_infer_kernel<false>, dim3(infer_grid(n)), dim3(kW), 0, s, n, pp, tv, tv, 0,
                     feat, m, scores);
  return hipGetLastError();
}

int policy_grad_waves(int n) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(n, 16))); }

hipError_t launch_policy_grad(const float* rec, const int32_t* idx, int n, const float* theta,
                              const PolicyNorm& nm, float* partial, int nwaves, float* grad, float* theta_out,
                              float* am, float* av, const PolicyAdam& ad, float* stats, hipStream_t s) {
  const int per = (int)ceil_div(std::max(n, 1), nwaves);
  hipLaunchKernelGGL(policy_grad_kernel, dim3((unsigned)nwaves), dim3(kW), 0, s, rec, idx, n, per, theta, nm,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(policy_reduce_kernel, dim3((unsigned)ceil_div(kPolicyParams + 1, 256)), dim3(256), 0, s,
                     partial, nwaves, grad, theta_out, am, av, ad, stats);
  return hipGetLastError();
}

}  // namespace gs
