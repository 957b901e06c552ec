// Expansion kernels: data layout and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs_internal.h"

namespace gs {

// Multi-index tables for the graded O(D^p) sets (section 2) up to order P,
// all in device memory.  Term index order: by degree, decreasing
// lexicographic inside a degree, so order p uses the first nterms[p] terms.
struct SeriesTables {
  int D = 0, P = 0, C = 0;
  const int8_t* alpha = nullptr;      // [C][D]
  const int32_t* deg = nullptr;       // [C]
  const double* inv_fact = nullptr;   // [C] 1/alpha!
  const int32_t* nterms = nullptr;    // [P+1] C(D+p-1, D)
  const int32_t* h2h_start = nullptr; // [C+1] per gamma: alpha <= gamma
  const int2* h2h_pairs = nullptr;    //   (alpha index, (gamma-alpha) index)
  const int32_t* l2l_start = nullptr; // [C+1] per alpha: beta >= alpha
  const int2* l2l_pairs = nullptr;    //   (beta index, (beta-alpha) index), beta ascending
  const double* l2l_coef = nullptr;   //   beta!/(alpha!(beta-alpha)!)
};

// Tree fields the expansion kernels read.
struct NodeView {
  const int32_t *begin, *count, *left;
  const double* ctr;  // [node][D]
  const double *lo, *hi;
};

// Sorted groups of one work type: run starts where key changes.
struct SortedGroups {
  int n = 0;
  const int4* grp = nullptr;             // unsorted group records {h, Q, first, n}
  const int32_t* order = nullptr;        // [n] group index in (h, Q, level) order
  const unsigned long long* key = nullptr;  // [n] sorted keys
};

hipError_t launch_p2m(const SeriesTables& T, const NodeView& t, int n_nodes, const double* xperm,
                      const double* wperm, double* M, hipStream_t s);
hipError_t launch_h2h_level(const SeriesTables& T, const NodeView& t, int lb, int le, double* M,
                            hipStream_t s);
// DH groups of one traversal level (their query nodes are disjoint per h).
hipError_t launch_dh_level(const SeriesTables& T, const int4* grp, int ng, int max_q, const int32_t* ent,
                           const NodeView& qt, const NodeView& rt, const double* xq_perm,
                           const double* M, const double* sc, int M_q, double* gdh, hipStream_t s);
hipError_t launch_dl(const SeriesTables& T, const SortedGroups& g, const int32_t* ent,
                     const NodeView& qt, const NodeView& rt, const double* xr_perm,
                     const double* wr_perm, const double* sc, int nQ, double* lco, int32_t* pL,
                     hipStream_t s);
hipError_t launch_h2l(const SeriesTables& T, const SortedGroups& g, const int32_t* ent,
                      const NodeView& qt, const NodeView& rt, const double* M, const double* sc,
                      int nQ, double* lco, int32_t* pL, hipStream_t s);
hipError_t launch_l2l_level(const SeriesTables& T, const NodeView& qt, int lb, int le, int n_h,
                            int nQ, const double* sc, double* lco, int32_t* pL, double* Gest,
                            hipStream_t s);
hipError_t launch_leaf_eval(const SeriesTables& T, const NodeView& qt, const int32_t* leaves,
                            int n_leaves, int n_h, int nQ, int M_q, const double* sc,
                            const double* xq_perm, const int32_t* qperm, const double* gx,
                            const double* gdh, const double* Gest, const double* lco,
                            const int32_t* pL, double* G_out, hipStream_t s);

// Compile-time specialisations of DH, DL, H2L and the post-pass for the
// order-limit table's (D, P) pairs, with graded (O(D^p)) or, with tensor,
// tensor (O(p^D)) index sets; launch_*_fast return hipErrorInvalidValue for
// other pairs.
bool series_fast_available(int D, int P, bool tensor);
//
// DH of one traversal level: slices[0..ns) {group, first entry, entries,
// slice of the group} of its groups grp[g0..g0+ng), first[g] = the global
// index of group g's first slice, slice0 = the global index of slices[0].
// max_q: an upper bound on the point count of the groups' query nodes.  A
// group of one slice adds into gdh directly; the slices of a longer group
// write part[slice][chunk][64] (ns * ceil(max_q / 64) * 64 doubles), summed
// in slice order by a second kernel.
hipError_t launch_dh_fast(int D, int P, bool tensor, const int4* slices, int ns, int slice0, const int4* grp,
                          const int32_t* first, int g0, int ng, int max_q, const int32_t* ent,
                          const NodeView& qt, const NodeView& rt, const double* xq_perm,
                          const double* M, const double* sc, int Mq, double* gdh, double* part,
                          hipStream_t s);
// DL of the whole traversal: slices[0..ns) {group, first chunk, end chunk}
// over each group's entries (cpre[entry] = chunks of the group's earlier
// entries), one partial coefficient vector per slice (part: ns * C doubles,
// part_p: ns orders), then per (h, Q) run of the sorted groups g the sum over
// its groups' slices (first[group] = {first slice, slices}) in order into lco.
hipError_t launch_dl_fast(int D, int P, bool tensor, const SortedGroups& g, const int4* slices, int ns,
                          const int2* first, const int32_t* cpre, const int32_t* ent,
                          const NodeView& qt, const NodeView& rt, const double* xr_perm,
                          const double* wr_perm, const double* sc, int nQ, double* lco, int32_t* pL,
                          double* part, int32_t* part_p, hipStream_t s);
// H2L of the whole traversal: one partial coefficient vector per group (part:
// groups * C doubles, part_p: groups orders), then per (h, Q) run of the
// sorted groups g their sum in order into lco.
hipError_t launch_h2l_fast(int D, int P, bool tensor, const SortedGroups& g, const int32_t* ent,
                           const NodeView& qt, const NodeView& rt, const double* M, const double* sc,
                           int nQ, double* lco, int32_t* pL, double* part, int32_t* part_p,
                           hipStream_t s);
// H2H of the internal nodes [lb, le) of one tree level, as launch_h2h_level.
hipError_t launch_h2h_level_fast(int D, int P, bool tensor, const NodeView& t, int lb, int le, double* M,
                                 hipStream_t s);
// Leaf moments (raw, h-independent) of every leaf node (internal nodes are
// left alone; H2H fills them), as launch_p2m.
hipError_t launch_p2m_fast(int D, int P, bool tensor, const NodeView& t, int n_nodes, const double* xperm,
                           const double* wperm, double* M, hipStream_t s);
// Size of the DL partial coefficient vectors (C(D+P-1, D), or P^D for tensor sets).
int series_terms(int D, int P, bool tensor);
// Post-pass in one launch (grid: query nodes x bandwidths, internal nodes
// exit): G_out[h][qperm[q]] = gx + gdh + sum over the leaf and its ancestors
// A (parent[], -1 at the root) of Gest_A + EVALL(lco_A, pL_A, x_q); lco may
// be null when every pL is 0.
hipError_t launch_leaf_post_fast(int D, int P, bool tensor, const NodeView& qt, const int32_t* parent, int nQ,
                                 int n_h, int Mq, const double* sc, const double* xq_perm,
                                 const int32_t* qperm, const double* gx, const double* gdh,
                                 const double* Gest, const double* lco, const int32_t* pL,
                                 double* G_out, hipStream_t s);

// Base cases (DITOBase), fused over blocks of kBaseHB bandwidths: a base
// entry is (Q, R, block) with the block's bandwidths that chose the base case
// in a kBaseHB-bit mask, so that one squared distance serves all of them.
constexpr int kBaseHB = 16;
typedef uint16_t BaseMask;
int base_record_stride(int D);

// Reference records for the base tiles: per leaf, its points' float
// coordinates relative to the leaf centre and weight / max weight, padded with
// zero records to a multiple of 4; rec_off[leaf] = the leaf's first record.
struct BaseRecordsArgs {
  const double* xr_perm = nullptr;  // [N][D], reference tree order
  const double* wr_perm = nullptr;
  const int32_t *leaf_of_pos = nullptr, *begin = nullptr, *count = nullptr, *left = nullptr;
  const double* rctr = nullptr;
  int64_t n = 0;
  int D = 0, n_nodes = 0;
  const unsigned long long* wmax_bits = nullptr;
  int32_t* padded = nullptr;   // [n_nodes] scratch
  int32_t* rec_off = nullptr;  // [n_nodes] out
  float* rec = nullptr;        // [rec_capacity][base_record_stride(D)] out
  int64_t rec_capacity = 0;
  // MFMA distance records (when base_uses_mfma(D); else mrec = nullptr): per
  // leaf, groups of 32 references [base_mfma_group_floats(D)] from
  // mgrp_off[leaf]; rmax2[leaf] = largest |x_r - c_leaf|^2 of its points
  float* mrec = nullptr;
  int64_t mgroups_capacity = 0;  // base_mfma_groups_capacity
  int32_t* mgrp_off = nullptr;   // [n_nodes] out
  float* rmax2 = nullptr;        // [n_nodes] out
  void* temp = nullptr;
  size_t temp_bytes = 0;
};
bool base_uses_mfma(int D);
int64_t base_mfma_groups_capacity(int64_t n_points, int n_nodes);
int base_mfma_group_floats(int D);
int64_t base_records_capacity(int64_t n_points, int n_nodes);
size_t base_records_temp_bytes(int n_nodes);
hipError_t launch_base_records(const BaseRecordsArgs& a, hipStream_t s);

struct BaseFusedArgs {
  // base work list of the traversal: groups {h, Q, first entry, entries}
  const int4* grp = nullptr;
  int n_groups = 0;
  const int32_t* ent = nullptr;  // (R << 4) | p
  int64_t n_entries = 0;
  int n_qnodes = 0, n_rnodes = 0, n_hblocks = 0;
  int max_leaf = 0;  // most points in a query leaf
  // bandwidths [hc0, hc1) are written by this call; others are left alone
  int hc0 = 0, hc1 = 0;
  NodeView qt{}, rt{};
  const double* xq_perm = nullptr;  // [M][D], query tree order
  const float* rec = nullptr;       // reference records (BaseRecordsArgs)
  const int32_t* rec_off = nullptr;
  const float* mrec = nullptr;      // MFMA distance records (BaseRecordsArgs; may be null)
  const int32_t* mgrp_off = nullptr;
  const float* rmax2 = nullptr;
  unsigned long long* mfma_evals = nullptr;  // += point-pair evaluations with MFMA distances
  int D = 0, Mq = 0;
  const float* s2 = nullptr;        // log2(e) / 2h^2 per bandwidth
  const unsigned long long* wmax_bits = nullptr;
  double* gx = nullptr;             // [n_h][M]
  unsigned long long* dist_evals = nullptr;  // += point pairs of the regrouped entries
  // scratch: n_entries elements each (run_start n_entries + 1)
  unsigned long long *key = nullptr, *key_sorted = nullptr, *ukey = nullptr;
  BaseMask *bit = nullptr, *bit_sorted = nullptr, *umask = nullptr;
  int32_t *flag = nullptr, *pos = nullptr, *mflag = nullptr, *mpos = nullptr, *run_start = nullptr;
  int4* slices = nullptr;    // base_max_slices(n_entries)
  int4* slots = nullptr;     // base_partial_slots(max_leaf)
  double* partial = nullptr; // base_partial_doubles(max_leaf)
  int32_t* counters = nullptr;  // 8: unique entries, runs, slices, partial slots used, slice queue
  int32_t* host_counters = nullptr;  // 4, page-locked host memory: the plan's readbacks
  void* temp = nullptr;
  size_t temp_bytes = 0;
};

struct BaseFusedPlan {
  int n_slices = 0, n_slots = 0, max_slots = 0, slice_entries = 0, qmax = 0, rbits = 0, hbits = 0;
};

size_t base_fused_temp_bytes(int64_t n_entries);
int64_t base_max_slices(int64_t n_entries);
int base_partial_slots(int max_leaf);
// doubles of the partial-sum array: slots * kBaseHB * round_up(max_leaf, 64)
int64_t base_partial_doubles(int max_leaf);
// Regroups the entries into runs and slices (synchronises the stream twice).
hipError_t plan_base_fused(const BaseFusedArgs& a, BaseFusedPlan* p, hipStream_t s);
hipError_t launch_base_fused(const BaseFusedArgs& a, const BaseFusedPlan& p, hipStream_t s);

}  // namespace gs
