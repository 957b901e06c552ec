// Learned pair policy: layout, device views and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "gs_internal.h"

namespace gs {

constexpr int kPolicyIn = 16, kPolicyHidden = 64, kPolicyOut = 4;
constexpr int kPolicyParams = kPolicyHidden * kPolicyIn + kPolicyHidden + kPolicyHidden * kPolicyHidden +
                              kPolicyHidden + kPolicyOut * kPolicyHidden + kPolicyOut;  // 5508
// A training record: features[16], targets[4] (log2 ns), masks[4].
constexpr int kPolicyRecord = kPolicyIn + 2 * kPolicyOut;
// Packed half-precision weight tiles (A-operand layout): W1 4, W2 16, W3 4.
constexpr int kPolicyTiles = 24;
// Normalisation stored after the parameters: mu_x[16], sd_x[16], mu_y, sd_y.
constexpr int kPolicyNormFloats = 2 * kPolicyIn + 2;

// Pairs of one frontier level: pair g belongs to segment seg[g] = (h, Q).
struct PolicyPairs {
  const int32_t *h = nullptr, *Q = nullptr, *seg = nullptr, *R = nullptr;
  const double *hs = nullptr, *invh = nullptr;  // per bandwidth: h and 1/h
};

struct PolicyTreeView {
  const double *lo = nullptr, *hi = nullptr, *rinf = nullptr;
  const int32_t *count = nullptr, *left = nullptr;
};

struct PolicyDevModel {
  const void* wpack = nullptr;  // kPolicyTiles x 64 lanes x 4 halves
  const float *b1 = nullptr, *b2 = nullptr, *b3 = nullptr;
  float mu_x[kPolicyIn], isd_x[kPolicyIn];
};

struct PolicyNorm {
  float mu_x[kPolicyIn], isd_x[kPolicyIn];
  float mu_y, isd_y;
};

struct PolicyAdam {
  float lr = 1e-3f, beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  float bc1 = 1.0f, bc2 = 1.0f;  // 1 - beta^step
};

hipError_t launch_policy_features(int npair, const PolicyPairs& pp, const PolicyTreeView& qt,
                                  const PolicyTreeView& rt, int D, float* feat, hipStream_t s);
hipError_t launch_policy_infer_pairs(int npair, const PolicyPairs& pp, const PolicyTreeView& qt,
                                     const PolicyTreeView& rt, int D, const PolicyDevModel& m,
                                     float4* scores, hipStream_t s);
hipError_t launch_policy_infer_features(int n, const float* feat, const PolicyDevModel& m, float4* scores,
                                        hipStream_t s);
// Waves of the gradient kernel for a batch of n records.
int policy_grad_waves(int n);
// grad (optional): mean gradient; theta_out (optional): Adam step in place
// (theta_out == theta).  partial: nwaves * (kPolicyParams + 2) floats.
// stats[2] = (loss, mask sum).
hipError_t launch_policy_grad(const float* rec, const int32_t* idx, int n, const float* theta,
                              const PolicyNorm& nm, float* partial, int nwaves, float* grad, float* theta_out,
                              float* am, float* av, const PolicyAdam& ad, float* stats, hipStream_t s);

// Host state of a context's policy.
struct PolicyState {
  bool ready = false;                 // parameters and normalisation set
  std::vector<float> theta;           // kPolicyParams
  float mu_x[kPolicyIn], sd_x[kPolicyIn];
  float mu_y = 0.0f, sd_y = 1.0f;
  bool dev_fresh = false;  // the workspace copies (pol_theta, pol_wpack) match theta
  // cost model, ns per unit
  double c_pair = 0.0, c_dh = 0.0, c_dl = 0.0, c_h2l = 0.0, c_base = 0.0;
  bool costs_pinned = false;  // set by the caller: logging does not recalibrate
  // training records of the last logged call, and their (h, level, Q, R)
  std::vector<float> log;
  std::vector<int32_t> log_keys;
};

}  // namespace gs
