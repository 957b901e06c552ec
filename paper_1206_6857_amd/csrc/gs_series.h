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

// Compile-time specialisations of DH and DL for the order-limit table's
// (D, P) pairs; launch_*_fast return hipErrorInvalidValue for other pairs.
bool series_fast_available(int D, int P);
// max_q: an upper bound on the point count of the groups' query nodes.
hipError_t launch_dh_fast(int D, int P, const int4* grp, int ng, int max_q, const int32_t* ent,
                          const NodeView& qt, const NodeView& rt, const double* xq_perm,
                          const double* M, const double* sc, int Mq, double* gdh, hipStream_t s);
hipError_t launch_dl_fast(int D, int P, const SortedGroups& g, const int32_t* ent,
                          const NodeView& qt, const NodeView& rt, const double* xr_perm,
                          const double* wr_perm, const double* sc, int nQ, double* lco, int32_t* pL,
                          hipStream_t s);

// Base cases (DITOBase): gx[h][q] for the runs of BASE groups.
int base_record_stride(int D);
hipError_t launch_base_records(const double* xr_perm, const double* wr_perm, const int32_t* leaf_of_pos,
                               const double* rctr, int64_t n, int D, const unsigned long long* wmax_bits,
                               float* rec, hipStream_t s);
hipError_t launch_base(const SortedGroups& g, const int32_t* ent, const NodeView& qt,
                       const NodeView& rt, const double* xq_perm, const float* rec, int D,
                       const float* s2, const unsigned long long* wmax_bits, int M_q, double* gx,
                       hipStream_t s);

}  // namespace gs
