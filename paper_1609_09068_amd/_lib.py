"""ctypes binding of libpr.so (include/pr.h).

Argument marshalling only: every step of the method runs in the library.
PyTorch supplies device memory (tensors' data pointers) and the HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpr.so")

PR_OK = 0
PR_NOT_CONVERGED = 1
PR_EINVAL = -1
PR_ENOMEM = -2
PR_EHIP = -3
PR_EHANDLE = -4

PR_METHOD_COMPONENTWISE = 0
PR_METHOD_PLAIN = 1
PR_STOP_CERT_L1 = 0
PR_STOP_PAPER_MAXABS = 1
PR_PREC_MIXED = 0
PR_PREC_FP64 = 1
PR_PREC_AUTO = 2


class BuildOpts(C.Structure):
    _fields_ = [("small_cutoff", C.c_int32), ("team_edges", C.c_int32), ("rows_per_wave", C.c_int32),
                ("build_plain", C.c_int32), ("autotune", C.c_int32), ("keep_loops", C.c_int32),
                ("seg_waves", C.c_int32), ("reserved", C.c_int32 * 5)]


class SolveOpts(C.Structure):
    _fields_ = [("method", C.c_int32), ("stop", C.c_int32), ("precision", C.c_int32),
                ("use_graph", C.c_int32), ("eps", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int64), ("warm_start", C.c_void_p), ("trace", C.c_int32),
                ("kernel_timing", C.c_int32), ("warm_scope", C.c_int32), ("small_direct", C.c_int32),
                ("tail_estimate", C.c_int32), ("refine", C.c_int32), ("cold", C.c_int32),
                ("gs_blocks", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("edge_iters", C.c_int64), ("iters_max", C.c_int64), ("iters_sum", C.c_int64),
                ("n_iterated", C.c_int64), ("n_not_converged", C.c_int64), ("ws_accepted", C.c_int64),
                ("ws_rejected", C.c_int64), ("cert_abs", C.c_double), ("r_sum", C.c_double),
                ("cert_rel", C.c_double), ("time_ms", C.c_double), ("vert_iters", C.c_int64),
                ("kernel_ms", C.c_double), ("kt_ms", C.c_double * 4), ("kt_count", C.c_int64 * 4),
                ("gang_edge_iters", C.c_int64), ("gang_vert_iters", C.c_int64),
                ("cert_trunc_rel", C.c_double), ("res_l1", C.c_double), ("refine_rounds", C.c_int32),
                ("precision_used", C.c_int32), ("reserved", C.c_int32 * 2)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("reserved", "kt_ms", "kt_count")}
        d["kt_ms"] = list(self.kt_ms)
        d["kt_count"] = list(self.kt_count)
        return d


class LevelsInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n", "m", "n_comp", "n_levels", "n_scc", "n_cac", "n_singleton", "v_scc", "v_cac",
        "v_singleton", "m_scc_internal", "m_cac_internal", "m_between", "n_items", "n_gangs",
        "n_gang_scc", "v_gang", "m_gang_internal", "m_gang_between", "n_phases", "n_hubs")] + [(k, C.c_int32) for k in ("rows_per_wave", "small_cutoff", "team_edges", "grid_wgs", "seg_waves",
                                                      "reserved_i32")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol include/pr.h declares
EXPORTS = ["pr_partition", "pr_partition_get", "pr_default_build_opts", "pr_build_levels", "pr_build_levels_weighted",
           "pr_levels_get_info", "pr_default_solve_opts", "pr_solve", "pr_levels_debug", "pr_free",
           "pr_last_error", "pr_version", "pr_mlp_create", "pr_mlp_set_params", "pr_mlp_get_params",
           "pr_mlp_predict", "pr_mlp_grad", "pr_mlp_grad_noalloc", "pr_mlp_train_step", "pr_mlp_save",
           "pr_mlp_load",
           "pr_warm_features", "pr_bandwidth_probe"]

_lib = None
_owners = None
_finalizing = False


def track(owner):
    """Register an object that owns a library handle, so that it is released
    at interpreter exit while the HIP runtime is still up."""
    global _owners
    import weakref

    if _owners is None:
        _owners = weakref.WeakSet()
    _owners.add(owner)


def _release_all():
    """atexit hook: free every live handle (plans and networks first, they
    hold device memory), then ignore later frees.  Without it a handle whose
    owner survives to interpreter teardown would call hipFree / hipGraph*Destroy
    from a finalizer after the runtime (or a profiler's tool library) has shut
    down."""
    global _finalizing
    if _owners is not None:
        live = list(_owners)
        for kind in ("Levels", "Mlp", "Partition"):
            for o in live:
                if type(o).__name__ == kind:
                    try:
                        o.free()
                    except Exception:
                        pass
    _finalizing = True


def finalizing():
    return _finalizing


def load():
    """Load libpr.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1609_09068_amd.build_lib` (there is no fallback)")
    lib = C.CDLL(LIB_PATH)
    import atexit

    atexit.register(_release_all)
    P, I32, I64, U32, VP = C.POINTER, C.c_int32, C.c_int64, C.c_uint32, C.c_void_p
    lib.pr_partition.argtypes = [I64, P(I64), P(I32), U32, P(VP)]
    lib.pr_partition.restype = I32
    lib.pr_partition_get.argtypes = [VP, P(I32), P(I32), P(C.c_uint8), P(I32), P(I64), P(I32)]
    lib.pr_partition_get.restype = I32
    lib.pr_default_build_opts.argtypes = [P(BuildOpts)]
    lib.pr_default_build_opts.restype = None
    lib.pr_build_levels.argtypes = [VP, I64, P(I64), P(I32), P(BuildOpts), VP, P(VP)]
    lib.pr_build_levels.restype = I32
    lib.pr_build_levels_weighted.argtypes = [VP, I64, P(I64), P(I32), P(C.c_double), P(BuildOpts), VP, P(VP)]
    lib.pr_build_levels_weighted.restype = I32
    lib.pr_levels_get_info.argtypes = [VP, P(LevelsInfo)]
    lib.pr_levels_get_info.restype = I32
    lib.pr_default_solve_opts.argtypes = [P(SolveOpts)]
    lib.pr_default_solve_opts.restype = None
    lib.pr_solve.argtypes = [VP, C.c_double, VP, VP, P(SolveOpts), VP, P(SolveStats)]
    lib.pr_solve.restype = I32
    lib.pr_levels_debug.argtypes = [VP, I32, VP]
    lib.pr_levels_debug.restype = I32
    lib.pr_free.argtypes = [VP]
    lib.pr_free.restype = None
    lib.pr_last_error.argtypes = []
    lib.pr_last_error.restype = C.c_char_p
    lib.pr_version.argtypes = []
    lib.pr_version.restype = C.c_char_p
    F32P, D = P(C.c_float), C.c_double
    lib.pr_mlp_create.argtypes = [C.c_uint64, P(VP)]
    lib.pr_mlp_set_params.argtypes = [VP, F32P]
    lib.pr_mlp_get_params.argtypes = [VP, F32P]
    lib.pr_mlp_predict.argtypes = [VP, I64, VP, VP, VP]
    lib.pr_mlp_grad.argtypes = [VP, I64, VP, VP, F32P, P(D), VP]
    lib.pr_mlp_grad_noalloc.argtypes = [VP, I64, VP, VP, F32P, P(D), VP]
    lib.pr_mlp_train_step.argtypes = [VP, I64, VP, VP, C.c_float, P(D), VP]
    lib.pr_mlp_save.argtypes = [VP, C.c_char_p]
    lib.pr_mlp_load.argtypes = [C.c_char_p, P(VP)]
    lib.pr_warm_features.argtypes = [VP, D, VP, VP, VP, VP, VP]
    lib.pr_bandwidth_probe.argtypes = [VP, I64, I32, VP, P(D)]
    lib.pr_bandwidth_probe.restype = I32
    for name in ("pr_mlp_create", "pr_mlp_set_params", "pr_mlp_get_params", "pr_mlp_predict", "pr_mlp_grad",
                 "pr_mlp_grad_noalloc",
                 "pr_mlp_train_step", "pr_mlp_save", "pr_mlp_load", "pr_warm_features"):
        getattr(lib, name).restype = I32
    _lib = lib
    return lib


class PRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc, allow=(PR_OK,)):
    if rc not in allow:
        raise PRError(rc, load().pr_last_error().decode())
    return rc


def _as_csr(row_ptr, col):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    return row_ptr, col


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))
