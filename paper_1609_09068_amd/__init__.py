"""Componentwise PageRank on MI355X (gfx950).

The SCC/CAC partition of Sec. 4.1 runs on the host (C++); the intermediate
step (Sec. 4.2) and the level-by-level PageRank step (Sec. 4.3) run in HIP
kernels.  Everything is reached through the C ABI of libpr.so (include/pr.h);
this module only marshals arguments.  torch tensors provide device buffers
and the stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from .weights import expand_integer_weights  # noqa: F401
from ._lib import (PR_METHOD_COMPONENTWISE, PR_METHOD_PLAIN, PR_PREC_AUTO, PR_PREC_FP64, PR_PREC_MIXED,  # noqa: F401
                   PR_STOP_CERT_L1, PR_STOP_PAPER_MAXABS, PRError, PR_NOT_CONVERGED)


class Partition:
    """Owner of a pr_partition_t handle (freed with the object)."""

    def __init__(self, handle, n):
        self.handle = handle
        self.n = n
        _lib.track(self)
        lib = _lib.load()
        k = C.c_int64()
        L = C.c_int32()
        _lib._check(lib.pr_partition_get(handle, None, None, None, None, C.byref(k), C.byref(L)))
        K = k.value
        self.n_comp = K
        self.n_levels = L.value
        self.comp = np.zeros(n, dtype=np.int32)
        self.comp_level = np.zeros(K, dtype=np.int32)
        self.comp_type = np.zeros(K, dtype=np.uint8)
        self.comp_size = np.zeros(K, dtype=np.int32)
        _lib._check(lib.pr_partition_get(handle, _lib._ptr(self.comp, C.c_int32),
                                         _lib._ptr(self.comp_level, C.c_int32),
                                         _lib._ptr(self.comp_type, C.c_uint8),
                                         _lib._ptr(self.comp_size, C.c_int32), None, None))

    def as_dict(self):
        return dict(comp=self.comp, comp_level=self.comp_level, comp_type=self.comp_type,
                    comp_size=self.comp_size, n_comp=self.n_comp, n_levels=self.n_levels)

    def free(self):
        if self.handle and not _lib.finalizing():
            _lib.load().pr_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Levels:
    """Owner of a pr_levels_t handle (the device plan)."""

    def __init__(self, handle, n):
        self.handle = handle
        self.n = n
        _lib.track(self)

    def info(self):
        inf = _lib.LevelsInfo()
        _lib._check(_lib.load().pr_levels_get_info(self.handle, C.byref(inf)))
        return inf.as_dict()

    def debug(self, what, n_comp=None):
        lib = _lib.load()
        if what == "wprime":
            out = np.zeros(self.n, dtype=np.float64)
            code = 0
        elif what == "iters":
            out = np.zeros(n_comp, dtype=np.int32)
            code = 1
        elif what == "perm":
            out = np.zeros(self.n, dtype=np.int32)
            code = 2
        elif what == "wgstats":
            out = np.zeros((self.info()["grid_wgs"], 16), dtype=np.uint64)
            code = 3
        elif what == "trace":
            out = np.zeros((self.info()["n_items"], 4), dtype=np.uint64)
            code = 4
        elif what == "items":
            out = np.zeros((self.info()["n_items"], 4), dtype=np.int32)
            code = 5
        elif what == "rank_vbeg":
            out = np.zeros(self.info()["n_comp"] + 1, dtype=np.int32)
            code = 6
        elif what == "rank_comp":
            out = np.zeros(self.info()["n_comp"], dtype=np.int32)
            code = 7
        else:
            raise ValueError(what)
        _lib._check(lib.pr_levels_debug(self.handle, code, out.ctypes.data_as(C.c_void_p)))
        return out

    def free(self):
        if self.handle and not _lib.finalizing():
            _lib.load().pr_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Mlp:
    """Owner of a pr_mlp_t handle: the starting-guess network."""

    N_PARAMS = 4545

    def __init__(self, handle):
        self.handle = handle
        _lib.track(self)

    @classmethod
    def create(cls, seed=0):
        h = C.c_void_p()
        _lib._check(_lib.load().pr_mlp_create(C.c_uint64(seed), C.byref(h)))
        return cls(h.value)

    @classmethod
    def load_file(cls, path):
        h = C.c_void_p()
        _lib._check(_lib.load().pr_mlp_load(str(path).encode(), C.byref(h)))
        return cls(h.value)

    def save(self, path):
        _lib._check(_lib.load().pr_mlp_save(self.handle, str(path).encode()))

    def get_params(self):
        out = np.zeros(self.N_PARAMS, dtype=np.float32)
        _lib._check(_lib.load().pr_mlp_get_params(self.handle, _lib._ptr(out, C.c_float)))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        if theta.shape != (self.N_PARAMS,):
            raise ValueError("expected 4545 parameters")
        _lib._check(_lib.load().pr_mlp_set_params(self.handle, _lib._ptr(theta, C.c_float)))

    def predict(self, X, stream=None):
        """X: float32 device tensor [n, 4]; returns a float32 device tensor [n]."""
        import torch

        _need_f32_dev(X, 2)
        y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _lib._check(_lib.load().pr_mlp_predict(self.handle, X.shape[0], C.c_void_p(X.data_ptr()),
                                               C.c_void_p(y.data_ptr()), C.c_void_p(_stream_ptr(stream))))
        return y

    def grad(self, X, t, stream=None):
        """Gradient of the mean squared error on (X, t); returns (grad [4545], loss)."""
        _need_f32_dev(X, 2)
        _need_f32_dev(t, 1)
        g = np.zeros(self.N_PARAMS, dtype=np.float32)
        loss = C.c_double()
        _lib._check(_lib.load().pr_mlp_grad(self.handle, X.shape[0], C.c_void_p(X.data_ptr()),
                                            C.c_void_p(t.data_ptr()), _lib._ptr(g, C.c_float), C.byref(loss),
                                            C.c_void_p(_stream_ptr(stream))))
        return g, loss.value

    def grad_noalloc(self, X, t, stream=None):
        """grad() through pr_mlp_grad_noalloc (partials in the library's static
        device array; nothing allocated)."""
        _need_f32_dev(X, 2)
        _need_f32_dev(t, 1)
        g = np.zeros(self.N_PARAMS, dtype=np.float32)
        loss = C.c_double()
        _lib._check(_lib.load().pr_mlp_grad_noalloc(self.handle, X.shape[0], C.c_void_p(X.data_ptr()),
                                                    C.c_void_p(t.data_ptr()), _lib._ptr(g, C.c_float),
                                                    C.byref(loss), C.c_void_p(_stream_ptr(stream))))
        return g, loss.value

    def train_step(self, X, t, lr, stream=None):
        _need_f32_dev(X, 2)
        _need_f32_dev(t, 1)
        loss = C.c_double()
        _lib._check(_lib.load().pr_mlp_train_step(self.handle, X.shape[0], C.c_void_p(X.data_ptr()),
                                                  C.c_void_p(t.data_ptr()), C.c_float(lr), C.byref(loss),
                                                  C.c_void_p(_stream_ptr(stream))))
        return loss.value

    def free(self):
        if self.handle and not _lib.finalizing():
            _lib.load().pr_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _need_f32_dev(x, dim):
    if not x.is_cuda or x.dtype.itemsize != 4 or not x.dtype.is_floating_point or x.dim() != dim \
            or not x.is_contiguous():
        raise TypeError(f"expected a contiguous float32 device tensor of dimension {dim}")
    if dim == 2 and x.shape[1] != 4:
        raise ValueError("features must have 4 columns")


def warm_features(levels: "Levels", c, W, stream=None):
    """Features, component scale and SCC mask of every vertex from the last solve
    of `levels` with weights W (see pr_warm_features)."""
    import torch

    n = levels.n
    F = torch.empty((n, 4), dtype=torch.float32, device=W.device)
    S = torch.empty(n, dtype=torch.float32, device=W.device)
    M = torch.empty(n, dtype=torch.uint8, device=W.device)
    _lib._check(_lib.load().pr_warm_features(levels.handle, float(c), C.c_void_p(W.data_ptr()),
                                             C.c_void_p(F.data_ptr()), C.c_void_p(S.data_ptr()),
                                             C.c_void_p(M.data_ptr()), C.c_void_p(_stream_ptr(stream))))
    return F, S, M


def pr_partition(row_ptr, col) -> Partition:
    row_ptr, col = _lib._as_csr(row_ptr, col)
    n = len(row_ptr) - 1
    h = C.c_void_p()
    _lib._check(_lib.load().pr_partition(n, _lib._ptr(row_ptr, C.c_int64), _lib._ptr(col, C.c_int32), 0,
                                         C.byref(h)))
    return Partition(h.value, n)


def build_opts(**kw):
    o = _lib.BuildOpts()
    _lib.load().pr_default_build_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def solve_opts(**kw):
    o = _lib.SolveOpts()
    _lib.load().pr_default_solve_opts(C.byref(o))
    for k, v in kw.items():
        if k == "warm_start":
            v = v.handle if v is not None and not isinstance(v, int) else v
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def pr_build_levels(part: Partition, row_ptr, col, stream=None, weight=None, **opts) -> Levels:
    """The solve plan; with `weight` (one float per edge, col order) the plan
    of the weighted graph (pr_build_levels_weighted)."""
    row_ptr, col = _lib._as_csr(row_ptr, col)
    n = len(row_ptr) - 1
    o = build_opts(**opts)
    h = C.c_void_p()
    lib = _lib.load()
    if weight is None:
        rc = lib.pr_build_levels(part.handle, n, _lib._ptr(row_ptr, C.c_int64), _lib._ptr(col, C.c_int32),
                                 C.byref(o), C.c_void_p(_stream_ptr(stream)), C.byref(h))
    else:
        w = np.ascontiguousarray(weight, dtype=np.float64)
        if w.shape != col.shape:
            raise ValueError(f"weight has shape {w.shape}, expected {col.shape}")
        rc = lib.pr_build_levels_weighted(part.handle, n, _lib._ptr(row_ptr, C.c_int64), _lib._ptr(col, C.c_int32),
                                          _lib._ptr(w, C.c_double), C.byref(o), C.c_void_p(_stream_ptr(stream)),
                                          C.byref(h))
    _lib._check(rc)
    return Levels(h.value, n)


def pr_solve(levels: Levels, c, W, R, stream=None, **opts):
    """W, R: float64 device tensors of length n (caller's vertex order).
    Returns (return code, stats dict); raises PRError on a negative code."""
    if W.dtype.itemsize != 8 or R.dtype.itemsize != 8 or not W.is_cuda or not R.is_cuda:
        raise TypeError("W and R must be float64 device tensors")
    if W.numel() != levels.n or R.numel() != levels.n:
        raise ValueError("W / R must have n entries")
    if not (W.is_contiguous() and R.is_contiguous()):
        raise ValueError("W / R must be contiguous")
    o = solve_opts(**opts)
    st = _lib.SolveStats()
    rc = _lib.load().pr_solve(levels.handle, float(c), C.c_void_p(W.data_ptr()), C.c_void_p(R.data_ptr()),
                              C.byref(o), C.c_void_p(_stream_ptr(stream)), C.byref(st))
    _lib._check(rc, allow=(_lib.PR_OK, _lib.PR_NOT_CONVERGED))
    return rc, st.as_dict()


def pr_free(obj):
    obj.free()


def pr_last_error() -> str:
    return _lib.load().pr_last_error().decode()


def version() -> str:
    return _lib.load().pr_version().decode()


def bandwidth_probe(buf, reps=20, stream=None):
    """Milliseconds per read pass over a device tensor (pr_bandwidth_probe)."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise TypeError("expected a contiguous device tensor")
    ms = C.c_double()
    _lib._check(_lib.load().pr_bandwidth_probe(C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(), reps,
                                               C.c_void_p(_stream_ptr(stream)), C.byref(ms)))
    return ms.value
