// Level-synchronous dual-tree traversal: device-side data layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_internal.h"

namespace gs {

// Largest frontier (pairs or segments) and work list (entries or groups) of
// one traversal: offsets are 32-bit.
constexpr int64_t kMaxFrontier = (int64_t)1 << 30;

// Per-call constants of the pruning test (sections 4-5).
struct DecideConst {
  int D = 0, P = 0;
  int mono = 0, use_tokens = 1, use_fmm = 1;
  int log_pairs = 0;
  int fmm_mask = 7;  // allowed series methods: bit 0 DH, bit 1 DL, bit 2 H2L
  int policy = 0;    // 1: choose by the scores of the learned policy
  int log_feas = 0;  // 1: record the admitted orders where bestMethod is reached
  int node_bounds = 0;  // 0: box distances; 1: the tighter of box and ball distances
  double explore = 0.0;  // logging: probability of taking the direct path
                         // instead of the rule's series choice
  double eps_alg = 0.0;
  // [2]: token deposits and withdrawals of the call's decisions, summed in
  // weight units (section 5: a negative need is a deposit); may be null
  double* tok = nullptr;
  int tensor = 0;  // 1: O(p^D) expansions (tensor index sets) and their bounds
  double bconst[kMaxPlimit + 1];  // C(D+p-1, D-1) / sqrt(F(p)), Lemma 4
  double binomD[kMaxPlimit + 1];  // C(D+p-1, D), Lemma 6
  // O(p^D) bounds: Cramer's constant, 1/sqrt(n!) and 1/sqrt(p+1)
  double kc = 0.0;
  double isf[kMaxPlimit + 1];
  double isq[kMaxPlimit + 1];
  // Figure 6's cost model, saturated at INT64_MAX: per-point cost of an
  // order-p expansion (D^(p+1), or D p^D for tensor sets) and of an order-p
  // H2L translation (D^(2p+1), or D p^(2D))
  int64_t cterm[kMaxPlimit + 1];
  int64_t ch2l[kMaxPlimit + 1];
};

// Counters of one frontier segment (one (bandwidth, query node) pair list).
struct SegCount {
  int64_t v[18];  // [0] next-level pairs, [1] next-level segments,
                  // [2..5] DH, DL, H2L, BASE entries, [6..9] group flags,
                  // [10] FD pairs, [11] SPLIT pairs, [12] base-case point
                  // pairs, [13] policy consultations, [14] policy overrides,
                  // [15] DH slices, [16] DL slices, [17] next-level
                  // segments of at least kLongSegment pairs
};

// Segments this long are listed first (FrontierLevel::first) and raise their
// wave's issue priority: the longest token walks start before the short ones.
constexpr int kLongSegment = 128;

struct FrontierLevel {
  int32_t *h = nullptr, *Q = nullptr, *off = nullptr, *len = nullptr;
  double *T = nullptr, *Lp = nullptr;
  int32_t* R = nullptr;    // pairs
  int32_t* seg = nullptr;  // segment of each pair
  int32_t* first = nullptr;  // the segments of at least kLongSegment pairs
};

// Node fields read by the decision kernel.
struct TreeView {
  const double *lo, *hi, *rinf, *W, *wmin;
  const int32_t *count, *left;
  const double *ctr = nullptr, *rad = nullptr;  // for the sphere-rectangle bounds
};

// Work list entries: (R << 4) | p; groups: {h, Q, first entry, entries}.
// Slices: DH {group, first entry, entries, slice of the group}, with
// dh_first[group] = its first slice; DL {group, first chunk, end chunk, 0},
// chunks counted over the group's entries in order, with dl_first[group] =
// {first slice, slices} and dl_cpre[entry] = chunks of the group's earlier
// entries.  Group and slice indices are global over the traversal.
struct WorkLists {
  int32_t* ent[4];
  int4* grp[4];
  int4* dh_slice;
  int32_t* dh_first;
  int4* dl_slice;
  int2* dl_first;
  int32_t* dl_cpre;
};

struct LevelOffsets {
  int32_t ent[4];
  int32_t grp[4];
  int32_t slc[2];  // DH, DL slices
};

// scores (policy): per pair of the level, predicted log2 costs of DH, DL,
// H2L, recurse.  feas (log_feas): per pair, 0x8000 | q_DH | q_DL << 4 |
// q_H2L << 8 (smallest admitted orders, 0 = none) where bestMethod is
// reached, else 0.
// n_first: entries of cur.first (every segment of at least kLongSegment pairs).
// prep: scratch of 5 * npair doubles (the pair prepass), npair: the level's
// pairs.
// Reorders every segment's pairs of the level in place (cur.R) by decreasing
// dmin^2, ties by increasing R; d2 and r_tmp are npair scratch elements.
hipError_t launch_far_first_order(int npair, const FrontierLevel& cur, const TreeView& qt, const TreeView& rt,
                                  int D, int node_bounds, double* d2, int32_t* r_tmp, hipStream_t s);

hipError_t launch_decide(int S, int n_first, const FrontierLevel& cur, const TreeView& qt, const TreeView& rt,
                         const double* inv2h2, const double* inv4h2, const double* invh, int nQ,
                         const DecideConst& c, int8_t* code, int8_t* porder, double* Gest,
                         SegCount* cnt, const float4* scores, int16_t* feas, double* prep,
                         int npair, hipStream_t s);

hipError_t scan_counts(int S, const SegCount* cnt, SegCount* incl, void* temp, size_t temp_bytes,
                       hipStream_t s);
size_t scan_counts_temp_bytes(int S);

// Also adds the level's decision counters: hcount[h * 6 + code] (pairs per
// bandwidth and code) and ev[0], ev[2], ev[3] (base-case point pairs, policy
// consultations, fallbacks), from the inclusive scan at the ends of each run
// of equal bandwidths, a few atomics per bandwidth.
hipError_t launch_emit(int S, const FrontierLevel& cur, const FrontierLevel& nxt,
                       const int32_t* qleft, const int32_t* rleft, const int8_t* code,
                       const int8_t* porder, const SegCount* cnt, const SegCount* incl,
                       const int32_t* rcount, const WorkLists& wl, LevelOffsets base,
                       unsigned long long* hcount, unsigned long long* ev, hipStream_t s);

}  // namespace gs
