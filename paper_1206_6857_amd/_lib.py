"""ctypes binding of libgausssum.so (include/gausssum.h).

Argument marshalling only: every computation runs in the HIP library.  If the
library has not been built, loading fails loudly; there is no fallback.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgausssum.so")

GS_OK, GS_EINVAL, GS_ENOMEM, GS_EDEVICE, GS_EOVERFLOW, GS_EINTERNAL = 0, -1, -2, -3, -4, -5
GS_DUALTREE, GS_EXHAUSTIVE, GS_DFD, GS_DFDO, GS_DFTO = 0, 1, 2, 3, 4
GS_RULE, GS_LEARNED = 0, 1
METHODS = {"dualtree": GS_DUALTREE, "dito": GS_DUALTREE, "exhaustive": GS_EXHAUSTIVE,
           "dfd": GS_DFD, "dfdo": GS_DFDO, "dfto": GS_DFTO}
POLICIES = {"rule": GS_RULE, "learned": GS_LEARNED}
GS_BOUNDS_BOX, GS_BOUNDS_SPHERE_RECT = 0, 1
NODE_BOUNDS = {"box": GS_BOUNDS_BOX, "sphere_rect": GS_BOUNDS_SPHERE_RECT}
GS_ORDER_TREE, GS_ORDER_FAR_FIRST = 0, 1
PAIR_ORDERS = {"tree": GS_ORDER_TREE, "far_first": GS_ORDER_FAR_FIRST}
STATUS_NAMES = {0: "GS_OK", -1: "GS_EINVAL", -2: "GS_ENOMEM", -3: "GS_EDEVICE",
                -4: "GS_EOVERFLOW", -5: "GS_EINTERNAL"}

# Every function the header declares; tests check that the library exports them.
EXPORTED = ["gs_default_options", "gs_create", "gs_destroy", "gauss_sum", "gs_get_stats",
            "gs_get_pair_counts", "gs_last_error", "gs_get_tree", "gs_get_trace",
            "gs_multi_indices", "gs_tensor_indices", "gs_decision_arith", "gs_default_train_opts", "gs_policy_set_cost_model",
            "gs_policy_get_cost_model", "gs_policy_get_log", "gs_policy_write_log",
            "gs_policy_train", "gs_policy_train_records", "gs_policy_gradient",
            "gs_policy_predict", "gs_policy_get_params", "gs_policy_set_params",
            "gs_policy_save", "gs_policy_load", "gs_lscv", "gs_exhaustive_noalloc"]
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

POLICY_PARAMS = 5508          # W1[64][16] b1[64] W2[64][64] b2[64] W3[4][64] b3[4]
POLICY_PARAM_FLOATS = 5542    # + mu_x[16] sd_x[16] mu_y sd_y
POLICY_RECORD = 24            # features[16] targets[4] masks[4]
POLICY_FEATURES = 16          # raw features per pair


class GsOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("plimit", ctypes.c_int32), ("method", ctypes.c_int32),
                ("policy", ctypes.c_int32), ("monochromatic", ctypes.c_int32),
                ("blocking", ctypes.c_int32), ("keep_trace", ctypes.c_int32),
                ("log_pairs", ctypes.c_int32), ("fmm_mask", ctypes.c_int32),
                ("kernel_timing", ctypes.c_int32), ("h_chunk", ctypes.c_int32),
                ("eps_round_share", ctypes.c_double), ("max_frontier", ctypes.c_int64),
                ("log_explore", ctypes.c_double), ("autotune", ctypes.c_int32),
                ("node_bounds", ctypes.c_int32), ("debug_fail_alloc", ctypes.c_int32),
                ("log_path", ctypes.c_char_p), ("pair_order", ctypes.c_int32)]


class GsCostModel(ctypes.Structure):
    _fields_ = [("pair_ns", ctypes.c_double), ("dh_ns", ctypes.c_double), ("dl_ns", ctypes.c_double),
                ("h2l_ns", ctypes.c_double), ("base_ns", ctypes.c_double)]


class GsTrainOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("steps", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("reinit", ctypes.c_int32), ("seed", ctypes.c_uint64), ("lr", ctypes.c_double)]


class GsStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("n_h", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("plimit", ctypes.c_int32),
                ("pairs", ctypes.c_int64 * 6), ("base_pair_evals", ctypes.c_int64),
                ("frontier_peak", ctypes.c_int64), ("policy_calls", ctypes.c_int64),
                ("policy_overrides", ctypes.c_int64),
                ("t_stage_ms", ctypes.c_double), ("t_tree_ms", ctypes.c_double),
                ("t_moments_ms", ctypes.c_double), ("t_traverse_ms", ctypes.c_double),
                ("t_work_ms", ctypes.c_double), ("t_post_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("k_ms", ctypes.c_double * 12),
                ("k_launches", ctypes.c_int64 * 12), ("base_dist_evals", ctypes.c_int64),
                ("h_chunks", ctypes.c_int32), ("tuned_leaf_size", ctypes.c_int32),
                ("tuned_method", ctypes.c_int32), ("autotune_trials", ctypes.c_int32),
                ("workspace_requests", ctypes.c_int64), ("p_hist", (ctypes.c_int64 * 16) * 3),
                ("tokens_deposited", ctypes.c_double), ("tokens_withdrawn", ctypes.c_double),
                ("pair_evals_per_s", ctypes.c_double), ("base_mfma_pair_evals", ctypes.c_int64)]
K_BASE, K_EXHAUSTIVE, K_DECIDE, K_SERIES, K_POST, K_TREE, K_MOMENTS, K_DH, K_DL, K_H2L = range(10)


_lib = None


def load():
    """Load libgausssum.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgausssum.so is not built (run __graft_entry__.build()); "
                           "there is no CPU fallback")
    # The library uses the system ROCm runtime; PyTorch ships its own.  When
    # both live in one process, PyTorch's must initialise first or it finds no
    # device, so initialise it before the library's first HIP call.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.gs_default_options.argtypes = [ctypes.POINTER(GsOptions)]
    lib.gs_default_options.restype = None
    lib.gs_create.argtypes = [ctypes.POINTER(P), i32, P]
    lib.gs_create.restype = i32
    lib.gs_destroy.argtypes = [P]
    lib.gs_destroy.restype = i32
    lib.gauss_sum.argtypes = [P, P, i64, P, P, i64, i32, P, i32, f64, P, ctypes.POINTER(GsOptions)]
    lib.gauss_sum.restype = i32
    lib.gs_get_stats.argtypes = [P, ctypes.POINTER(GsStats)]
    lib.gs_get_stats.restype = i32
    lib.gs_get_pair_counts.argtypes = [P, P]
    lib.gs_get_pair_counts.restype = i32
    lib.gs_last_error.argtypes = [P]
    lib.gs_last_error.restype = ctypes.c_char_p
    lib.gs_get_tree.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)] + [P] * 11
    lib.gs_get_tree.restype = i32
    lib.gs_get_trace.argtypes = [P, ctypes.POINTER(i64), P]
    lib.gs_get_trace.restype = i32
    lib.gs_multi_indices.argtypes = [i32, i32, ctypes.POINTER(i64), P]
    lib.gs_multi_indices.restype = i32
    lib.gs_tensor_indices.argtypes = [i32, i32, ctypes.POINTER(i64), P]
    lib.gs_tensor_indices.restype = i32
    lib.gs_decision_arith.argtypes = [P, P, P, i64, P]
    lib.gs_decision_arith.restype = i32
    lib.gs_lscv.argtypes = [P, P, i64, i32, P, i32, f64, P, P, ctypes.POINTER(GsOptions)]
    lib.gs_lscv.restype = i32
    lib.gs_exhaustive_noalloc.argtypes = [P, P, i64, P, P, i64, i32, P, i32, P]
    lib.gs_exhaustive_noalloc.restype = i32
    pf = ctypes.POINTER(ctypes.c_float)
    lib.gs_default_train_opts.argtypes = [ctypes.POINTER(GsTrainOpts)]
    lib.gs_default_train_opts.restype = None
    lib.gs_policy_set_cost_model.argtypes = [P, ctypes.POINTER(GsCostModel)]
    lib.gs_policy_get_cost_model.argtypes = [P, ctypes.POINTER(GsCostModel)]
    lib.gs_policy_get_log.argtypes = [P, ctypes.POINTER(i64), P, P]
    lib.gs_policy_write_log.argtypes = [P, ctypes.c_char_p]
    lib.gs_policy_train.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(GsTrainOpts), pf]
    lib.gs_policy_train_records.argtypes = [P, P, i64, ctypes.POINTER(GsTrainOpts), pf]
    lib.gs_policy_gradient.argtypes = [P, P, i64, P, pf]
    lib.gs_policy_predict.argtypes = [P, P, i64, P]
    lib.gs_policy_get_params.argtypes = [P, P, i64]
    lib.gs_policy_set_params.argtypes = [P, P, i64]
    lib.gs_policy_save.argtypes = [P, ctypes.c_char_p]
    lib.gs_policy_load.argtypes = [P, ctypes.c_char_p]
    for name in ("gs_policy_set_cost_model", "gs_policy_get_cost_model", "gs_policy_get_log",
                 "gs_policy_write_log", "gs_policy_train", "gs_policy_train_records",
                 "gs_policy_gradient", "gs_policy_predict", "gs_policy_get_params",
                 "gs_policy_set_params", "gs_policy_save", "gs_policy_load"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib
