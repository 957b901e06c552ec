/*
 * gausssum.h - C ABI of the MI355X (gfx950) Gaussian summation library.
 *
 * Computes, for every query point x_q and every bandwidth h in a list,
 *
 *     G_h(x_q) = sum_{r=1}^{N} w_r exp(-|x_q - x_r|^2 / (2 h^2))
 *
 * (Lee & Gray, "Faster Gaussian Summation: Theory and Experiment", section 1),
 * either exhaustively or with the dual-tree algorithm of sections 5-6, which
 * guarantees |G~(x_q) - G(x_q)| <= eps G(x_q) for every query (Theorem 2).
 *
 * Conventions for every entry point:
 *   - Nothing is thrown across the ABI; every call returns a gs_status.
 *   - The caller owns all input and output buffers.  The library never keeps
 *     a caller pointer after a call returns.
 *   - Array pointers may point to host memory or to device memory of the
 *     context's device; the library inspects each pointer.  Host inputs are
 *     copied to the device inside the call; a host output is written back
 *     before the call returns.
 *   - A failed call leaves outputs unspecified and the context reusable; the
 *     reason is available from gs_last_error().  A failed gauss_sum or
 *     gs_lscv returns only after the work it had enqueued has finished, so
 *     the caller may free its buffers at once.
 *   - A context is not thread safe: calls on one context must not overlap.
 */
#ifndef GAUSSSUM_H
#define GAUSSSUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_ctx gs_ctx;
typedef int32_t gs_status;

enum {
  GS_OK = 0,
  GS_EINVAL = -1,     /* invalid argument or input value */
  GS_ENOMEM = -2,     /* device or host allocation failed */
  GS_EDEVICE = -3,    /* a HIP runtime call failed */
  GS_EOVERFLOW = -4,  /* a size exceeds what the library can index */
  GS_EINTERNAL = -5   /* internal consistency check failed */
};

/* Summation method (section 7 names the dual-tree variants). */
enum {
  GS_DUALTREE = 0,    /* finite difference + O(D^p) expansions + token rule (DITO) */
  GS_EXHAUSTIVE = 1,  /* all M*N terms, no tree */
  GS_DFD = 2,         /* finite difference only, local pruning rule (no tokens) */
  GS_DFDO = 3,        /* finite difference only, with the token rule of section 5 */
  GS_DFTO = 4         /* finite difference + O(p^D) expansions (every alpha_d < p) +
                         token rule.  The paper takes their error bounds from earlier
                         work; this library derives them from Cramer's inequality and
                         the product form of the tensor sets (per dimension a kept
                         part K a_p and a dropped part K b_p, telescoped over the D
                         factors, times exp(-dmin^2/4h^2) with the box distance).
                         Default order limit: the plimit table lowered until
                         p^D <= 286.  Needs node_bounds = GS_BOUNDS_BOX and
                         policy = GS_RULE; no log_pairs. */
};

/* How the series method is chosen for a node pair (Figure 6). */
enum {
  GS_RULE = 0,        /* the paper's cost model */
  GS_LEARNED = 1      /* the learned pair policy: it chooses among the actions the
                         error bound admits, so every choice is certified */
};

typedef struct gs_options {
  int32_t struct_size;      /* sizeof(gs_options); set by gs_default_options */
  int32_t leaf_size;        /* max points per kd-tree leaf (default 64, 1..1024) */
  int32_t plimit;           /* max expansion order; <= 0 selects the section 6
                               table (D=2:8, 3:6, 5:4, 6:2, >6:1) */
  int32_t method;           /* GS_DUALTREE, GS_EXHAUSTIVE, GS_DFD, GS_DFDO, GS_DFTO */
  int32_t policy;           /* GS_RULE or GS_LEARNED */
  int32_t monochromatic;    /* -1: auto (queries == refs and M == N), 0: no, 1: yes */
  int32_t blocking;         /* 1 (default): return after the results are written;
                               0: device outputs may still be in flight on the
                               context's stream when the call returns */
  int32_t keep_trace;       /* 1: keep the trees and the per-pair decision trace for
                               gs_get_tree / gs_get_trace (slow; for testing) */
  int32_t log_pairs;        /* 1: record policy-training features and costs */
  int32_t fmm_mask;         /* series methods bestMethod may choose (Figure 6): bit 0
                               DH, bit 1 DL, bit 2 H2L; 0 or 7 allows all (ablations) */
  int32_t kernel_timing;    /* 1: time every kernel class with HIP events on the stream
                               it runs on (gs_stats.k_ms / k_launches); 2: time only
                               the base-case tiles (GS_K_BASE) and the exhaustive
                               tiles (one event pair per call); 0: none */
  int32_t h_chunk;          /* most bandwidths traversed together (0: all); the
                               library halves it by itself when a frontier outgrows
                               2^30 pairs or device memory.  Results do not depend
                               on it beyond floating-point summation order. */
  double eps_round_share;   /* share of eps reserved for floating-point rounding
                               (default 0.1); the pruning test uses (1-share)*eps */
  int64_t max_frontier;     /* cap on the node pairs of one frontier level (bounds the
                               traversal's memory; 0: 2^30).  A chunk of bandwidths whose
                               frontier exceeds it is retried with half the bandwidths;
                               GS_EOVERFLOW when one bandwidth alone exceeds it. */
  double log_explore;       /* with log_pairs: share (0..1, default 0) of the pairs
                               reaching bestMethod whose action is drawn uniformly
                               from the admitted ones (each admitted series method
                               at its order, or the direct path) instead of the
                               rule's, so that the log also holds costs the rule
                               never incurs.  log_pairs needs policy = GS_RULE. */
  int32_t autotune;         /* 1: choose the leaf size (32..256) and, for GS_DUALTREE,
                               between the dual-tree and the exhaustive path, by timing
                               each once per workload signature (dimension, sizes, the
                               bandwidth range, eps, method options); the choice is
                               cached in the context.  Ignored with keep_trace. */
  int32_t node_bounds;      /* GS_BOUNDS_BOX (default): node-pair distance bounds from
                               the bounding boxes (section 5); GS_BOUNDS_SPHERE_RECT:
                               the tighter of those and the bounds from the nodes'
                               bounding balls about the box centres */
  int32_t debug_fail_alloc; /* error-path testing: k > 0 makes the k-th device
                               workspace request of the call (cached or not,
                               counted from 1 across the whole call) fail as an
                               out-of-memory would, so the call returns GS_ENOMEM
                               from wherever that request sits; the context stays
                               usable.  0 (default): off */
  const char* log_path;     /* with log_pairs: also write the call's training records
                               to this file (gs_policy_write_log's format; read by
                               gs_policy_train) before returning; NULL (default): keep
                               them in the context only (gs_policy_get_log).  The
                               library does not keep the pointer. */
  int32_t pair_order;       /* the order in which the token walk takes a query node's
                               reference list at each level: GS_ORDER_TREE (default:
                               left to right, the order of the recursion of Figure 1)
                               or GS_ORDER_FAR_FIRST (a best-first order in the spirit
                               of the priority-queue traversal of section 1: decreasing
                               squared box distance (with node_bounds, the tighter
                               bound), ties by reference node, so that far prunings
                               deposit their tokens before near pairs spend them) */
} gs_options;

enum { GS_BOUNDS_BOX = 0, GS_BOUNDS_SPHERE_RECT = 1 };
enum { GS_ORDER_TREE = 0, GS_ORDER_FAR_FIRST = 1 };

typedef struct gs_stats {
  int32_t struct_size;      /* set by the caller to sizeof(gs_stats) */
  int32_t n_h;              /* bandwidths in the last call */
  int32_t levels;           /* frontier levels of the last traversal */
  int32_t plimit;           /* expansion order limit used */
  int64_t pairs[6];         /* resolved node pairs over all h: FD, DH, DL, H2L,
                               BASE, and SPLIT decisions */
  int64_t base_pair_evals;  /* point-pair kernel evaluations in base cases */
  int64_t frontier_peak;    /* largest frontier (pairs over all h) */
  int64_t policy_calls;     /* pairs on which the learned policy was consulted */
  int64_t policy_overrides; /* of those, pairs whose cheapest predicted action of all
                               four the bound did not admit, so the cheapest predicted
                               admitted one was taken.  The rule never takes over: the
                               policy only chooses among admitted actions. */
  double t_stage_ms, t_tree_ms, t_moments_ms, t_traverse_ms, t_work_ms, t_post_ms;
  double t_total_ms;        /* wall time of the last gauss_sum call */
  /* With kernel_timing (1: all classes, 2: GS_K_BASE and GS_K_EXHAUSTIVE only): device
   * milliseconds and launch counts per kernel class,
   * indexed by GS_K_*. */
  double k_ms[12];
  int64_t k_launches[12];
  int64_t base_dist_evals;  /* point pairs whose squared distance the base tiles
                               formed (one per pair for all bandwidths of a block) */
  int32_t h_chunks;         /* bandwidth chunks the traversal was split into */
  int32_t tuned_leaf_size;  /* leaf size the call used */
  int32_t tuned_method;     /* method the call used (the autotuner may pick GS_EXHAUSTIVE) */
  int32_t autotune_trials;  /* timed trial runs this call made (0: cached or off) */
  int64_t workspace_requests; /* device workspace requests the call made (cached or
                               not; the range of gs_options.debug_fail_alloc) */
  int64_t p_hist[3][16];    /* dual-tree calls: node pairs resolved by DH, DL and H2L
                               (first index) at each order p (second index, 1..plimit;
                               Figure 6's chosen orders) over all bandwidths */
  double tokens_deposited;  /* token rule (section 5), over all bandwidths and query
                               nodes, in weight units: the sum of the token gains of
                               the decisions (base cases add W_R, approximations whose
                               need W E/(eps L) - W_R is negative add -need) ... */
  double tokens_withdrawn;  /* ... and the sum of the positive needs the approximations
                               spent.  Summed with atomics: the last bits can differ
                               between identical calls. */
  double pair_evals_per_s;  /* M N n_h / t_total_ms: the call's rate in point-pair
                               evaluations per second equivalent (section 7's measure
                               of a whole sweep, preprocessing included) */
  int64_t base_mfma_pair_evals; /* of base_pair_evals, those whose squared distance came
                               from the matrix cores (the norm expansion, admitted per
                               leaf pair and bandwidth where its rounding stays below
                               2^-12 of a term); the rest use the difference form */
} gs_stats;

/* Kernel classes of gs_stats.k_ms. */
enum {
  GS_K_BASE = 0,        /* base-case tiles */
  GS_K_EXHAUSTIVE = 1,  /* plain exhaustive tiles */
  GS_K_DECIDE = 2,      /* frontier decisions, policy inference, scan and emission */
  GS_K_SERIES = 3,      /* DH, DL and H2L work together */
  GS_K_POST = 4,        /* L2L and leaf evaluation */
  GS_K_TREE = 5,        /* tree construction */
  GS_K_MOMENTS = 6,     /* leaf moments and H2H */
  GS_K_DH = 7,          /* of GS_K_SERIES: direct Hermite evaluation */
  GS_K_DL = 8,          /* of GS_K_SERIES: direct local accumulation */
  GS_K_H2L = 9          /* of GS_K_SERIES: Hermite-to-local translation */
};

/* Fill *opt with the defaults listed above. */
void gs_default_options(gs_options* opt);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run on
 * (for example torch's current stream), or NULL to let the context create its
 * own stream.  The context owns its device workspace. */
gs_status gs_create(gs_ctx** out, int32_t device, void* hip_stream);

/* Free the context and its workspace.  NULL is a no-op. */
gs_status gs_destroy(gs_ctx* ctx);

/* Multi-bandwidth Gaussian summation (section 1) to relative error eps per query
 * (Theorem 2).
 *   queries    [M][D] row-major doubles; may equal `refs` (monochromatic: each
 *              query also receives its own term w_q)
 *   refs       [N][D] row-major doubles
 *   weights    [N] doubles, each > 0 (section 1 requires w_r > 0)
 *   bandwidths [n_h] doubles, each > 0
 *   eps        relative error tolerance, 0 < eps < 1 (ignored by GS_EXHAUSTIVE)
 *   G_out      [n_h][M] doubles in the caller's query order
 *   opt        options, or NULL for defaults
 * Errors: GS_EINVAL for M, N, n_h < 1, D < 1 or D > 64, any NaN or infinite
 * coordinate, any weight <= 0, any bandwidth <= 0, eps outside (0,1), or an
 * option out of range. */
gs_status gauss_sum(gs_ctx* ctx, const double* queries, int64_t M, const double* refs,
                    const double* weights, int64_t N, int32_t D, const double* bandwidths,
                    int32_t n_h, double eps, double* G_out, const gs_options* opt);

/* Statistics of the last gauss_sum call.  out->struct_size must be set. */
gs_status gs_get_stats(gs_ctx* ctx, gs_stats* out);

/* Per-bandwidth node-pair counts of the last dual-tree call: counts[n_h][6] in
 * the order FD, DH, DL, H2L, BASE, SPLIT (host pointer). */
gs_status gs_get_pair_counts(gs_ctx* ctx, int64_t* counts);

/* Message describing the last non-OK status on this context; owned by the
 * context and valid until its next call. */
const char* gs_last_error(gs_ctx* ctx);

/* kd-tree of the last call made with keep_trace = 1 (section 6, Figure 5).
 * which: 0 = reference tree, 1 = query tree (the same tree when monochromatic).
 * All pointers are host pointers and may be NULL to skip a field; first call
 * with everything NULL to read *n_nodes and *n_points.
 *   perm[n_points]   original point index at each tree position
 *   begin/count/left[n_nodes]  point range and left child (-1 for a leaf; the
 *                    right child is left+1); nodes are numbered breadth first
 *   lo/hi/ctr[n_nodes][D], rinf/W/wmin[n_nodes] as defined in the tree builder
 *   rad[n_nodes]     Euclidean radius about ctr (computed when the call used
 *                    node_bounds = GS_BOUNDS_SPHERE_RECT, else 0) */
gs_status gs_get_tree(gs_ctx* ctx, int32_t which, int64_t* n_nodes, int64_t* n_points,
                      int32_t* perm, int32_t* begin, int32_t* count, int32_t* left, double* lo,
                      double* hi, double* ctr, double* rinf, double* W, double* wmin, double* rad);

/* Decision trace of the last call made with keep_trace = 1: one record per
 * decided node pair, int32 [n][6] = (bandwidth index, level, Q node, R node,
 * code, order p) with code 0 FD, 1 DH, 2 DL, 3 H2L, 4 base case, 5 split
 * (Figure 7).  records may be NULL to read *n_records first. */
gs_status gs_get_trace(gs_ctx* ctx, int64_t* n_records, int32_t* records);

/* ---------------------------------------------------------------------------
 * Learned pair policy.
 *
 * bestMethod (section 6, Figure 6) chooses among DH, DL, H2L and the direct
 * path (base case or split) with an operation-count model whose cut-offs the
 * paper calls rough.  With policy = GS_LEARNED a small network predicts, from
 * the pair's geometry only, the log2 cost in nanoseconds of four actions: DH,
 * DL and H2L at the smallest order their bound admits, and "recurse", the
 * cost-to-go of the direct path.  The cheapest predicted of the admitted
 * actions is taken: a series method is admitted where its error bound admits
 * an order (Lemmas 4-6, the test the rule uses), recursion always.  Theorem 2
 * therefore holds whatever the network predicts.
 *
 * Network: 16 features -> 64 ReLU -> 64 ReLU -> 4 outputs.  Parameter vector
 * (float, 5508): W1[64][16], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]; in
 * gs_policy_get_params / gs_policy_set_params it is followed by the
 * standardisation mu_x[16], sd_x[16], mu_y, sd_y (5542 floats in all): the
 * network sees (x - mu_x) / sd_x and predicts (log2 cost - mu_y) / sd_y.
 *
 * Training record (float[24]): features[16], targets[4] (log2 ns), masks[4]
 * (1 where the target is known).  Features of a pair (Q, R) at bandwidth h:
 * log2 N_Q, log2 N_R, log2(1 + dmin/h), log2(1 + dmax/h), log2 h,
 * log2(1 + rinf_Q/h), log2(1 + rinf_R/h), [Q is a leaf], [R is a leaf], D/16,
 * then six zeros.  Costs follow gs_cost_model: every decided pair costs
 * pair_ns, plus N_Q C(D+p-1,D) dh_ns (DH), N_R C dl_ns (DL), C^2 h2l_ns (H2L),
 * N_Q N_R base_ns (base case), or its children's cost-to-go (split).
 *
 * Callers: gauss_sum with log_pairs = 1 (and keep_trace implied) records one
 * training record per pair that reaches bestMethod; gs_policy_train* fits the
 * network with the library's own gradient and Adam kernels; gauss_sum with
 * policy = GS_LEARNED uses it.
 * ------------------------------------------------------------------------- */

typedef struct gs_cost_model {
  double pair_ns;   /* deciding one node pair */
  double dh_ns;     /* per query point and term of a direct Hermite evaluation */
  double dl_ns;     /* per reference point and term of a direct local accumulation */
  double h2l_ns;    /* per (term x term) of a Hermite-to-local translation */
  double base_ns;   /* per point pair of a base case */
} gs_cost_model;

typedef struct gs_train_opts {
  int32_t struct_size;  /* sizeof(gs_train_opts); set by gs_default_train_opts */
  int32_t steps;        /* Adam steps (default 3000) */
  int32_t batch;        /* records per step (default 4096; all if fewer) */
  int32_t reinit;       /* 1 (default): new standardisation from the records and
                           fresh parameters from seed; 0: continue from the
                           current parameters */
  uint64_t seed;        /* parameter initialisation and batch order (default 1) */
  double lr;            /* Adam learning rate (default 2e-3; betas 0.9, 0.999) */
} gs_train_opts;

void gs_default_train_opts(gs_train_opts* opts);

/* Cost model of the policy's training targets (defaults: measured on one
 * MI355X).  Each logging call (log_pairs = 1) first recalibrates the
 * work-type costs (dh, dl, h2l, base) from its own kernel timings, every one
 * whose kernels ran for at least 0.05 ms; pair_ns is kept, since a logging
 * call decides pairs at a higher cost than a plain one.  A model set here is
 * kept as given.  All fields must be >= 0. */
gs_status gs_policy_set_cost_model(gs_ctx* ctx, const gs_cost_model* cm);
gs_status gs_policy_get_cost_model(gs_ctx* ctx, gs_cost_model* cm);

/* Training records of the last gauss_sum call made with log_pairs = 1:
 * records[n][24] and keys[n][4] = (bandwidth index, level, Q, R), host
 * pointers, either may be NULL; call with both NULL to read *n_records. */
gs_status gs_policy_get_log(gs_ctx* ctx, int64_t* n_records, float* records, int32_t* keys);

/* Writes those records to a file (binary, this library's format). */
gs_status gs_policy_write_log(gs_ctx* ctx, const char* path);

/* Trains the policy on the records of a log file (gs_policy_write_log) or of
 * an array records[n][24] (host or device).  *final_loss (may be NULL): the
 * masked mean squared error over all records, in standardised units.
 * GS_EINVAL for n < 1, steps < 0, batch < 1, lr <= 0. */
gs_status gs_policy_train(gs_ctx* ctx, const char* log_path, const gs_train_opts* opts,
                          float* final_loss);
gs_status gs_policy_train_records(gs_ctx* ctx, const float* records, int64_t n,
                                  const gs_train_opts* opts, float* final_loss);

/* Gradient of the masked mean squared error at the current parameters over
 * records[n][24] (host or device): grad[5508] (host or device), *loss. */
gs_status gs_policy_gradient(gs_ctx* ctx, const float* records, int64_t n, float* grad,
                             float* loss);

/* Network outputs for raw features[n][16]: scores[n][4], standardised units
 * (host or device pointers; the half-precision inference kernel). */
gs_status gs_policy_predict(gs_ctx* ctx, const float* features, int64_t n, float* scores);

/* Parameters and standardisation, 5542 floats (host pointers; n must be 5542). */
gs_status gs_policy_get_params(gs_ctx* ctx, float* params, int64_t n);
gs_status gs_policy_set_params(gs_ctx* ctx, const float* params, int64_t n);

/* Parameter file with the cost model (binary, this library's format). */
gs_status gs_policy_save(gs_ctx* ctx, const char* path);
gs_status gs_policy_load(gs_ctx* ctx, const char* path);

/* Least-squares cross-validation score of the Gaussian kernel density
 * estimate of points[N][D] (the bandwidth-selection criterion of the
 * experiments, section 7), for every bandwidth:
 *   LSCV(h) = integral of f_h^2 - (2/N) sum_i f_{h,-i}(x_i)
 *           = (4 pi h^2)^(-D/2)/N^2 sum_i G_{sqrt2 h}(x_i)
 *             - 2 (2 pi h^2)^(-D/2)/(N(N-1)) sum_i (G_h(x_i) - 1),
 * with G the multi-bandwidth sum of the points against themselves, unit
 * weights (one gauss_sum sweep over h and sqrt(2) h).  scores[n_h] and, if
 * not NULL, bounds[n_h] (host or device): |score - exact| <= bound, from the
 * per-query guarantee of Theorem 2 (eps; 1e-3 for GS_EXHAUSTIVE's float
 * tiles).  opt as for gauss_sum (monochromatic is implied; keep_trace and
 * log_pairs are rejected).  GS_EINVAL for N < 2, n_h outside [1, 2048], a
 * bandwidth <= 0, or any gauss_sum argument error. */
gs_status gs_lscv(gs_ctx* ctx, const double* points, int64_t N, int32_t D, const double* bandwidths,
                  int32_t n_h, double eps, double* scores, double* bounds, const gs_options* opt);

/* Multi-index set of the O(D^p) expansions (section 2): every alpha with
 * |alpha| < p, ordered by degree and, inside a degree, in decreasing
 * lexicographic order (for D = 2, p = 2: (0,0), (1,0), (0,1)).  Writes
 * *n_terms = C(D+p-1, D) and, if alpha is not NULL, alpha[n_terms][D] (host
 * pointer).  GS_EINVAL unless 1 <= D <= 64 and 1 <= p <= 10. */
gs_status gs_multi_indices(int32_t D, int32_t p, int64_t* n_terms, int32_t* alpha);

/* Multi-index set of the O(p^D) expansions of GS_DFTO (section 2): every alpha
 * with alpha_d < p in each dimension, ordered by the largest component and,
 * for one largest component, in decreasing lexicographic order, so that the
 * set of order p is the first p^D entries of any larger order (for D = 2,
 * p = 2: (0,0), (1,1), (1,0), (0,1)).  Writes *n_terms = p^D and, if alpha is
 * not NULL, alpha[n_terms][D] (host pointer).  GS_EINVAL unless 1 <= D <= 64,
 * 1 <= p <= 10 and p^D <= 286. */
gs_status gs_tensor_indices(int32_t D, int32_t p, int64_t* n_terms, int32_t* alpha);

/* The FP64 operations every pruning decision is made of (the token rule of
 * section 5 and bestMethod of Figure 6 compare bounds formed from them),
 * evaluated on the device exactly as the decide kernels do: out[0][i] = the
 * library's own exp(x[i]) (Cody-Waite reduction, degree-13 Taylor polynomial;
 * 0 below -700), out[1][i] = x[i] / y[i], out[2][i] = sqrt(y[i]).  Host
 * pointers x[n], y[n], out[3][n]; 1 <= n <= 2^24, else GS_EINVAL.  Tests
 * compare these bits with the host's correctly rounded division and square
 * root and with an independent exp of the same definition.  Its device buffers
 * are freed before it returns. */
gs_status gs_decision_arith(gs_ctx* ctx, const double* x, const double* y, int64_t n, double* out);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * gs_exhaustive_noalloc computes what gauss_sum computes with method =
 * GS_EXHAUSTIVE (the plain sum of section 1 over all M*N pairs, same kernels,
 * same launch configuration, bit-identical results) but makes no device
 * allocation: no hipMalloc, no hipFree, no allocating library call.  Its
 * intermediates (a validation flag, the largest weight, float reference
 * records, partial sums per reference split) live in one fixed device array
 * of the library of GS_NOALLOC_SCRATCH_BYTES, which every device the library
 * runs on holds until the process ends.
 *   queries [M][D], refs [N][D], weights [N], G_out [n_h][M]: device pointers
 *            on the context's device (queries may equal refs); the caller
 *            allocates them
 *   bandwidths [n_h]: host pointer
 * The call runs on the context's stream and returns after the results are
 * written (it reads back one validation flag before the sum).
 * Scratch needed: 256 + 4 N ceil((2D+1)/4)*4 bytes of records (each rounded
 * up to 256) + 8 S n_h M bytes of partial sums, where S, the reference
 * splits, is at most 1 + 2048 / ceil(M/256); so S M <= 524288 + M.
 * Errors: GS_EINVAL as for gauss_sum (sizes, NaN or infinite coordinates,
 * weights <= 0, bandwidths <= 0) and when an array is not where stated;
 * GS_EOVERFLOW when the call needs more scratch than the array holds (the
 * message gives both sizes).  Every call on one device shares that device's
 * array and leaves the last call's contents in it: calls that overlap on one
 * device (two contexts, two threads, or two streams) race and must be
 * serialised by the caller. */
#define GS_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

gs_status gs_exhaustive_noalloc(gs_ctx* ctx, const double* queries, int64_t M, const double* refs,
                                const double* weights, int64_t N, int32_t D,
                                const double* bandwidths, int32_t n_h, double* G_out);

#ifdef __cplusplus
}
#endif

#endif /* GAUSSSUM_H */
