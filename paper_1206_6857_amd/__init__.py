"""MI355X (gfx950) multi-bandwidth Gaussian summation (Lee & Gray, "Faster
Gaussian Summation: Theory and Experiment").

Python binding of the C ABI in include/gausssum.h.  The functions here only
marshal arguments: all arithmetic runs in the HIP library libgausssum.so.
Arrays may be NumPy arrays (host) or torch tensors (host or device); torch is
used only for device memory and streams.
"""

import ctypes

import numpy as np

from . import _lib
from ._lib import (GS_DFD, GS_DFDO, GS_DFTO, GS_DUALTREE, GS_EXHAUSTIVE, GS_LEARNED, GS_RULE,  # noqa: F401
                   GsOptions, GsStats)


class GaussSumError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_lib.STATUS_NAMES.get(status, status), message))
        self.status = status


def gs_default_options():
    opt = GsOptions()
    _lib.load().gs_default_options(ctypes.byref(opt))
    return opt


def _numel(a):
    n = 1
    for k in a.shape:
        n *= int(k)
    return n


def _rows(a, width, what):
    """Check that a marshalled array is [n][width]; returns n.  The library
    reads and writes exactly these sizes, so a mismatch would run past the
    caller's buffer."""
    if len(a.shape) != 2 or a.shape[1] != width:
        raise ValueError("%s must be [n][%d], got shape %s" % (what, width, a.shape))
    return a.shape[0]


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class _Arr:
    """Pointer to a contiguous float64 buffer (NumPy or torch), kept alive."""

    def __init__(self, x, writable=False):
        if _is_torch(x):
            import torch
            if x.dtype != torch.float64:
                raise TypeError("tensors must be float64")
            if not x.is_contiguous():
                raise ValueError("tensors must be contiguous")
            self.obj, self.ptr, self.is_cuda = x, x.data_ptr(), x.is_cuda
        else:
            a = np.asarray(x)
            if writable:
                if a.dtype != np.float64 or not a.flags.c_contiguous:
                    raise TypeError("output arrays must be C-contiguous float64")
            else:
                a = np.ascontiguousarray(a, dtype=np.float64)
            self.obj, self.ptr, self.is_cuda = a, a.ctypes.data, False
        self.shape = tuple(x.shape)


class Context:
    """Owns a gs_ctx: device workspace and a HIP stream (gs_create/gs_destroy)."""

    def __init__(self, device=0, stream=None):
        lib = _lib.load()
        h = ctypes.c_void_p()
        st = lib.gs_create(ctypes.byref(h), int(device), stream)
        if st != 0:
            raise GaussSumError(st, "gs_create failed on device %d" % device)
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().gs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return _lib.load().gs_last_error(self._h).decode()

    def _check(self, st):
        if st != 0:
            raise GaussSumError(st, self.last_error())

    def gauss_sum(self, queries, refs, weights, bandwidths, eps, out=None, **opts):
        """G[n_h][M] = sum_r w_r exp(-|q - r|^2 / 2h^2) to relative error eps.
        queries may be the same object as refs (monochromatic).  Options:
        method ('dualtree', 'exhaustive', 'dfd', 'dfdo', 'dfto'), policy ('rule',
        'learned'), leaf_size, plimit, monochromatic, eps_round_share,
        keep_trace, log_pairs, log_path, log_explore, blocking, fmm_mask,
        kernel_timing, h_chunk, max_frontier, node_bounds ('box', 'sphere_rect'),
        pair_order ('tree', 'far_first'), autotune, debug_fail_alloc."""
        lib = _lib.load()
        same = queries is refs
        r = _Arr(refs)
        q = r if same else _Arr(queries)
        w = _Arr(weights)
        hsrc = bandwidths
        if not _is_torch(hsrc):
            hsrc = np.atleast_1d(np.asarray(hsrc, dtype=np.float64))
        hb = _Arr(hsrc)
        if len(r.shape) != 2 or len(q.shape) != 2:
            raise ValueError("queries and refs must be 2-D [n][D]")
        M, D = q.shape
        N = r.shape[0]
        n_h = int(np.prod(hb.shape)) if hb.shape else 1
        if r.shape[1] != D:
            raise ValueError("queries and refs must have the same dimension (%d, %d)" % (D, r.shape[1]))
        if _numel(w) != N:
            raise ValueError("weights must hold one value per reference point (%d, got %d)" % (N, _numel(w)))
        if out is None:
            if q.is_cuda or r.is_cuda:
                import torch
                out = torch.empty((n_h, M), dtype=torch.float64, device=(q.obj if q.is_cuda else r.obj).device)
            else:
                out = np.empty((n_h, M), dtype=np.float64)
        o = _Arr(out, writable=True)
        if tuple(o.shape) != (n_h, M):
            raise ValueError("out must have shape (%d, %d), got %s" % (n_h, M, tuple(o.shape)))
        opt = gs_default_options()
        for k, v in opts.items():
            if k == "method":
                v = _lib.METHODS[v] if isinstance(v, str) else int(v)
            elif k == "policy":
                v = _lib.POLICIES[v] if isinstance(v, str) else int(v)
            elif k == "node_bounds":
                v = _lib.NODE_BOUNDS[v] if isinstance(v, str) else int(v)
            elif k == "pair_order":
                v = _lib.PAIR_ORDERS[v] if isinstance(v, str) else int(v)
            elif k == "log_path" and v is not None:
                v = str(v).encode()
            if not hasattr(opt, k):
                raise TypeError("unknown option %r" % k)
            setattr(opt, k, v)
        if any(a.is_cuda for a in (q, r, w, hb, o)):
            import torch
            torch.cuda.current_stream().synchronize()
        st = lib.gauss_sum(self._h, q.ptr, M, r.ptr, w.ptr, N, D, hb.ptr, n_h, float(eps), o.ptr,
                           ctypes.byref(opt))
        self._check(st)
        return out

    def exhaustive_noalloc(self, queries, refs, weights, bandwidths, out):
        """gs_exhaustive_noalloc: the exhaustive sum with no device allocation
        by the library.  queries, refs, weights and out are float64 device
        tensors (out [n_h][M]); bandwidths a host array."""
        lib = _lib.load()
        same = queries is refs
        r = _Arr(refs)
        q = r if same else _Arr(queries)
        w = _Arr(weights)
        hb = _Arr(np.atleast_1d(np.asarray(bandwidths, dtype=np.float64)))
        o = _Arr(out, writable=True)
        if len(r.shape) != 2 or len(q.shape) != 2:
            raise ValueError("queries and refs must be 2-D [n][D]")
        M, D = q.shape
        N = r.shape[0]
        n_h = hb.shape[0]
        if r.shape[1] != D:
            raise ValueError("queries and refs must have the same dimension (%d, %d)" % (D, r.shape[1]))
        if _numel(w) != N:
            raise ValueError("weights must hold one value per reference point (%d, got %d)" % (N, _numel(w)))
        if tuple(o.shape) != (n_h, M):
            raise ValueError("out must have shape (%d, %d), got %s" % (n_h, M, tuple(o.shape)))
        import torch
        torch.cuda.current_stream().synchronize()
        self._check(lib.gs_exhaustive_noalloc(self._h, q.ptr, M, r.ptr, w.ptr, N, D, hb.ptr, n_h, o.ptr))
        return out

    def stats(self):
        s = GsStats()
        s.struct_size = ctypes.sizeof(GsStats)
        self._check(_lib.load().gs_get_stats(self._h, ctypes.byref(s)))
        return s

    def pair_counts(self, n_h):
        out = np.zeros((n_h, 6), dtype=np.int64)
        self._check(_lib.load().gs_get_pair_counts(self._h, out.ctypes.data))
        return out

    def get_tree(self, which, D):
        """Tree arrays of the last call made with keep_trace=1 (gs_get_tree)."""
        lib = _lib.load()
        nn, npnt = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib.gs_get_tree(self._h, which, ctypes.byref(nn), ctypes.byref(npnt), *([None] * 11)))
        n, p = nn.value, npnt.value
        t = {"perm": np.zeros(p, np.int32), "begin": np.zeros(n, np.int32),
             "count": np.zeros(n, np.int32), "left": np.zeros(n, np.int32),
             "lo": np.zeros((n, D)), "hi": np.zeros((n, D)), "ctr": np.zeros((n, D)),
             "rinf": np.zeros(n), "W": np.zeros(n), "wmin": np.zeros(n), "rad": np.zeros(n)}
        order = ["perm", "begin", "count", "left", "lo", "hi", "ctr", "rinf", "W", "wmin", "rad"]
        self._check(lib.gs_get_tree(self._h, which, ctypes.byref(nn), ctypes.byref(npnt),
                                    *[t[k].ctypes.data for k in order]))
        return t

    def lscv(self, points, bandwidths, eps=0.01, **opts):
        """Least-squares cross-validation scores and error bounds (gs_lscv)
        of the Gaussian KDE of `points` for every bandwidth."""
        lib = _lib.load()
        x = _Arr(points)
        if len(x.shape) != 2:
            raise ValueError("points must be 2-D [n][D]")
        hsrc = bandwidths
        if not _is_torch(hsrc):
            hsrc = np.atleast_1d(np.asarray(hsrc, dtype=np.float64))
        hb = _Arr(hsrc)
        n_h = int(np.prod(hb.shape))
        N, D = x.shape
        scores = np.zeros(n_h)
        bounds = np.zeros(n_h)
        opt = gs_default_options()
        for k, v in opts.items():
            if k == "method":
                v = _lib.METHODS[v] if isinstance(v, str) else int(v)
            elif k == "policy":
                v = _lib.POLICIES[v] if isinstance(v, str) else int(v)
            if not hasattr(opt, k):
                raise TypeError("unknown option %r" % k)
            setattr(opt, k, v)
        if x.is_cuda or hb.is_cuda:
            import torch
            torch.cuda.current_stream().synchronize()
        self._check(lib.gs_lscv(self._h, x.ptr, N, D, hb.ptr, n_h, float(eps), scores.ctypes.data,
                                bounds.ctypes.data, ctypes.byref(opt)))
        return scores, bounds

    # ---- learned pair policy (gs_policy_*) ----

    def policy_log(self):
        """(records[n][24], keys[n][4]) of the last call made with log_pairs=1."""
        lib = _lib.load()
        n = ctypes.c_int64()
        self._check(lib.gs_policy_get_log(self._h, ctypes.byref(n), None, None))
        rec = np.zeros((n.value, _lib.POLICY_RECORD), dtype=np.float32)
        keys = np.zeros((n.value, 4), dtype=np.int32)
        self._check(lib.gs_policy_get_log(self._h, ctypes.byref(n), rec.ctypes.data, keys.ctypes.data))
        return rec, keys

    def policy_write_log(self, path):
        self._check(_lib.load().gs_policy_write_log(self._h, str(path).encode()))

    @staticmethod
    def _train_opts(**kw):
        o = _lib.GsTrainOpts()
        _lib.load().gs_default_train_opts(ctypes.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError("unknown training option %r" % k)
            setattr(o, k, v)
        return o

    def policy_train(self, records=None, log_path=None, **kw):
        """Fit the policy network (library kernels); returns the final loss."""
        lib = _lib.load()
        o = self._train_opts(**kw)
        loss = ctypes.c_float()
        if log_path is not None:
            self._check(lib.gs_policy_train(self._h, str(log_path).encode(), ctypes.byref(o),
                                            ctypes.byref(loss)))
        else:
            rec = np.ascontiguousarray(records, dtype=np.float32)
            _rows(rec, _lib.POLICY_RECORD, "records")
            self._check(lib.gs_policy_train_records(self._h, rec.ctypes.data, rec.shape[0],
                                                    ctypes.byref(o), ctypes.byref(loss)))
        return loss.value

    def policy_gradient(self, records):
        rec = np.ascontiguousarray(records, dtype=np.float32)
        _rows(rec, _lib.POLICY_RECORD, "records")
        g = np.zeros(_lib.POLICY_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        self._check(_lib.load().gs_policy_gradient(self._h, rec.ctypes.data, rec.shape[0], g.ctypes.data,
                                                   ctypes.byref(loss)))
        return g, loss.value

    def policy_predict(self, features):
        f = np.ascontiguousarray(features, dtype=np.float32)
        _rows(f, _lib.POLICY_FEATURES, "features")
        out = np.zeros((f.shape[0], 4), dtype=np.float32)
        self._check(_lib.load().gs_policy_predict(self._h, f.ctypes.data, f.shape[0], out.ctypes.data))
        return out

    def policy_params(self):
        out = np.zeros(_lib.POLICY_PARAM_FLOATS, dtype=np.float32)
        self._check(_lib.load().gs_policy_get_params(self._h, out.ctypes.data, out.size))
        return out

    def policy_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(_lib.load().gs_policy_set_params(self._h, p.ctypes.data, p.size))

    def policy_cost_model(self, **kw):
        """Get (no arguments) or update the cost model: pair_ns, dh_ns, dl_ns,
        h2l_ns, base_ns."""
        lib = _lib.load()
        cm = _lib.GsCostModel()
        self._check(lib.gs_policy_get_cost_model(self._h, ctypes.byref(cm)))
        if kw:
            for k, v in kw.items():
                if not hasattr(cm, k):
                    raise TypeError("unknown cost %r" % k)
                setattr(cm, k, float(v))
            self._check(lib.gs_policy_set_cost_model(self._h, ctypes.byref(cm)))
        return {k: getattr(cm, k) for k, _ in cm._fields_}

    def policy_save(self, path):
        self._check(_lib.load().gs_policy_save(self._h, str(path).encode()))

    def policy_load(self, path):
        self._check(_lib.load().gs_policy_load(self._h, str(path).encode()))

    def decision_arith(self, x, y):
        """(own exp(x), x / y, sqrt(y)) as the decide kernels compute them
        (gs_decision_arith), for equal-length float64 arrays x, y."""
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        y = np.ascontiguousarray(y, dtype=np.float64).ravel()
        if x.shape != y.shape:
            raise ValueError("x and y must have the same length")
        out = np.zeros((3, x.size), dtype=np.float64)
        self._check(_lib.load().gs_decision_arith(self._h, x.ctypes.data, y.ctypes.data, x.size,
                                                  out.ctypes.data))
        return out[0], out[1], out[2]

    def get_trace(self):
        """Decision records (h, level, Q, R, code, p) of the last keep_trace call."""
        lib = _lib.load()
        n = ctypes.c_int64()
        self._check(lib.gs_get_trace(self._h, ctypes.byref(n), None))
        rec = np.zeros((n.value, 6), dtype=np.int32)
        self._check(lib.gs_get_trace(self._h, ctypes.byref(n), rec.ctypes.data))
        return rec


def gs_multi_indices(D, p):
    """Library's multi-index set with |alpha| < p (host-side table; no GPU)."""
    lib = _lib.load()
    n = ctypes.c_int64()
    st = lib.gs_multi_indices(int(D), int(p), ctypes.byref(n), None)
    if st != 0:
        raise GaussSumError(st, "invalid D or p")
    out = np.zeros((n.value, D), dtype=np.int32)
    lib.gs_multi_indices(int(D), int(p), ctypes.byref(n), out.ctypes.data)
    return out


def gs_tensor_indices(D, p):
    """Library's O(p^D) multi-index set (every alpha_d < p; host-side table; no GPU)."""
    lib = _lib.load()
    n = ctypes.c_int64()
    st = lib.gs_tensor_indices(int(D), int(p), ctypes.byref(n), None)
    if st != 0:
        raise GaussSumError(st, "invalid D or p")
    out = np.zeros((n.value, D), dtype=np.int32)
    lib.gs_tensor_indices(int(D), int(p), ctypes.byref(n), out.ctypes.data)
    return out


_default = {}


def default_context(device=0):
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def gauss_sum(queries, refs, weights, bandwidths, eps, out=None, device=0, **opts):
    """Module-level gauss_sum on a per-device default context."""
    return default_context(device).gauss_sum(queries, refs, weights, bandwidths, eps, out=out, **opts)
