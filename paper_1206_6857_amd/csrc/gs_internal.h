// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace gs {

// Decision codes of a node pair (Figure 7): finite difference, direct Hermite
// evaluation, direct local accumulation, Hermite-to-local, base case, split.
enum PairCode : int32_t { FD = 0, DH = 1, DL = 2, H2L = 3, BASE = 4, SPLIT = 5 };

constexpr int kMaxD = 64;
constexpr int kMaxPlimit = 10;
constexpr int kMaxTerms = 286;      // C(D+p-1, D) bound enforced by the host
constexpr int kMaxHBlock = 16;      // bandwidths fused per exhaustive pass

// Slices of the series work lists, so that one long group spreads over many
// waves: a DH group's entries in runs of kDHSliceEntries, a DL group's point
// chunks (64 reference points, entry after entry) in runs of kDLSliceChunks.
constexpr int kDHSliceEntries = 8;
constexpr int kDLSliceChunks = 16;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- staging
hipError_t launch_stage_points(const double* x_rowmajor, int64_t n, int D, double* x_soa,
                               double* x_aos, int* bad_flag, hipStream_t s);
hipError_t launch_check_positive(const double* v, int64_t n, int* bad_flag, hipStream_t s);
// Raises bit 0 of *bad_flag if any of v[n] is NaN or infinite.
hipError_t launch_check_finite(const double* v, int64_t n, int* bad_flag, hipStream_t s);
// dst[i][d] = src[perm[i]][d];  dst[i] = src[perm[i]];  *out_bits = bits of max(w) (w > 0).
hipError_t launch_gather_rows(const double* src, const int32_t* perm, int64_t n, int D, double* dst,
                              hipStream_t s);
hipError_t launch_gather(const double* src, const int32_t* perm, int64_t n, double* dst,
                         hipStream_t s);
hipError_t launch_max_positive(const double* w, int64_t n, unsigned long long* out_bits,
                               hipStream_t s);

// ------------------------------------------------------------- exhaustive
// Records of split-precision reference coordinates: [hi_0..hi_{D-1}, lo_0..lo_{D-1},
// w, pad] floats, stride rec_stride.
int exhaustive_record_stride(int D);
// wmax_bits receives the largest weight (bit pattern of a positive double).
hipError_t launch_exhaustive_records(const double* x_aos, const double* w, int64_t n, int D,
                                     float* rec, unsigned long long* wmax_bits, hipStream_t s);
// partial[n_split][n_h][M]; G_out[n_h][M].  The first is an upper bound for
// any D, the second the exact count launch_exhaustive uses for this D.
size_t exhaustive_partial_elems(int64_t M, int64_t N, int n_h);
size_t exhaustive_partial_elems_exact(int64_t M, int64_t N, int D, int n_h);
hipError_t launch_exhaustive(const double* xq_aos, int64_t M, const float* rec, int64_t N, int D,
                             const double* bandwidths_host, int n_h,
                             const unsigned long long* wmax_bits, double* partial, double* G_out,
                             hipStream_t s);

// ------------------------------------------------------------------- LSCV
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
// sums[r] = sum_i G[r][i] (fixed order), for r < rows.
hipError_t launch_lscv_reduce(const double* G, int rows, int64_t N, double* sums, hipStream_t s);
// score/bound[n_h] from sums[2 n_h] (h rows, then sqrt(2) h rows) and hs[n_h] (device).
hipError_t launch_lscv_combine(const double* sums, const double* hs, int n_h, int64_t N, int D, double eps,
                               double* score, double* bound, hipStream_t s);

}  // namespace gs
