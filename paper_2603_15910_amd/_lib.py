"""ctypes declarations of the libcqk C ABI (include/cqk.h).

Only marshalling lives here: every computation runs in the HIP library.  A
missing library raises ``CqkLibraryMissing``; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcqk.so")

CQK_OK = 0
CQK_INFEASIBLE = 1
CQK_INVALID_ARG = 2
CQK_NOT_CONVERGED = 3
CQK_DEVICE_ERROR = 4
CQK_NO_MEMORY = 5
CQK_BUFFER_TOO_SMALL = 6
CQK_NOALLOC_MAX_SEG = 65536   # rows the no-allocation batched call holds
CQK_THETA_CANDIDATES = 7      # the theta tuner's candidates
THETA_CANDIDATES = (0.2, 0.3, 0.4, 0.5, 0.6, 0.75, 1.0)
STATUS_NAMES = {0: "OK", 1: "INFEASIBLE", 2: "INVALID_ARG", 3: "NOT_CONVERGED",
                4: "DEVICE_ERROR", 5: "NO_MEMORY", 6: "BUFFER_TOO_SMALL"}

LAMBDA0 = {"zero": 0, "formula": 1, "condat": 2, "user": 3}
COMPACTION = {"off": 0, "auto": 1, "always": 2}
ACCUM = {"default": 0, "f32": 1, "f64": 2}


class CqkLibraryMissing(RuntimeError):
    pass


class cqk_opts(C.Structure):
    _fields_ = [
        ("lambda0_mode", C.c_int32),
        ("lambda0_user", C.c_double),
        ("max_iter", C.c_int32),
        ("tol", C.c_double),
        ("compaction", C.c_int32),
        ("compact_theta", C.c_double),
        ("accum", C.c_int32),
        ("sync", C.c_int32),
        ("trace", C.c_int32),
        ("timing", C.c_int32),
    ]


class cqk_info(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("iterations", C.c_int32),
        ("passes", C.c_int32),
        ("stop_reason", C.c_int32),
        ("lambda_", C.c_double),
        ("lambda0", C.c_double),
        ("residual", C.c_double),
        ("abs_bx", C.c_double),
        ("n_free", C.c_int64),
        ("n_after_init", C.c_int64),
        ("pass_bytes", C.c_double),
        ("pass_ms", C.c_double),
        ("finalize_bytes", C.c_double),
        ("finalize_ms", C.c_double),
        ("rows_spilled", C.c_int64),
        ("pass_launches", C.c_int64),
    ]

    def as_dict(self):
        d = {f[0]: getattr(self, f[0]) for f in self._fields_}
        d["lambda"] = d.pop("lambda_")
        d["status_name"] = STATUS_NAMES.get(d["status"], str(d["status"]))
        return d


class cqk_trace_rec(C.Structure):
    _fields_ = [
        ("iter", C.c_int32),
        ("kind", C.c_int32),
        ("compacted", C.c_int32),
        ("source", C.c_int32),
        ("lam", C.c_double),
        ("phi", C.c_double),
        ("slope", C.c_double),
        ("lo", C.c_double),
        ("hi", C.c_double),
        ("n_in", C.c_int64),
        ("n_out", C.c_int64),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class cqk_batch_schedule(C.Structure):
    _fields_ = [
        ("small_per", C.c_int32),
        ("blocks_per_cu", C.c_int32),
        ("short_first", C.c_int32),
        ("medium_tiles", C.c_int32),
    ]

    def as_dict(self):
        return {f[0]: getattr(self, f[0]) for f in self._fields_}


class cqk_spg_opts(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("max_iter", C.c_int32),
        ("memory", C.c_int32),
        ("warm", C.c_int32),
        ("pad_", C.c_int32),
    ]


class cqk_spg_info(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("iterations", C.c_int32),
        ("projections", C.c_int64),
        ("newton_iterations", C.c_int64),
        ("objective", C.c_double),
        ("pg", C.c_double),
        ("total_ms", C.c_double),
        ("proj_ms", C.c_double),
    ]

    def as_dict(self):
        d = {f[0]: getattr(self, f[0]) for f in self._fields_}
        d["status_name"] = STATUS_NAMES.get(d["status"], str(d["status"]))
        return d


_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_D = C.c_double
_OPTS = C.POINTER(cqk_opts)
_INFO = C.POINTER(cqk_info)

# name -> (restype, argtypes); the same list as include/cqk.h
SIGNATURES = {
    "cqk_create": (C.c_int, [C.POINTER(_P), _P]),
    "cqk_destroy": (None, [_P]),
    "cqk_set_stream": (C.c_int, [_P, _P]),
    "cqk_reserve": (C.c_int, [_P, _I64, _I32]),
    "cqk_status_string": (C.c_char_p, [_I32]),
    "cqk_default_opts": (None, [_OPTS]),
    "cqk_last_trace": (C.c_int, [_P, C.POINTER(cqk_trace_rec), _I32, C.POINTER(_I32)]),
    "cqk_last_pass_ms": (C.c_int, [_P, C.POINTER(C.c_float), _I32, C.POINTER(_I32)]),
    "cqk_ctx_last_info": (C.c_int, [_P, _INFO]),
    "cqk_solve_f64": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_solve_f32": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_simplex_f32": (C.c_int, [_P, _I64, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_simplex_f64": (C.c_int, [_P, _I64, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_l1_f32": (C.c_int, [_P, _I64, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_l1_f64": (C.c_int, [_P, _I64, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_simplex_sparse_f32": (C.c_int, [_P, _I64, _P, _P, _D, _I64, _P, _P, _P, _OPTS,
                                                 _INFO]),
    "cqk_project_simplex_sparse_f64": (C.c_int, [_P, _I64, _P, _P, _D, _I64, _P, _P, _P, _OPTS,
                                                 _INFO]),
    "cqk_project_l1_sparse_f32": (C.c_int, [_P, _I64, _P, _P, _D, _I64, _P, _P, _P, _OPTS, _INFO]),
    "cqk_project_l1_sparse_f64": (C.c_int, [_P, _I64, _P, _P, _D, _I64, _P, _P, _P, _OPTS, _INFO]),
    "cqk_solve_batched_f64": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                        _OPTS, _INFO]),
    "cqk_solve_batched_backward_f64": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P,
                                                 _P, _OPTS]),
    "cqk_solve_batched_f32": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                        _OPTS, _INFO]),
    "cqk_solve_batched_backward_f32": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P,
                                                 _P, _OPTS]),
    "cqk_spg_default_opts": (None, [C.POINTER(cqk_spg_opts)]),
    "cqk_spg_l1_lasso_f64": (C.c_int, [_P, _I64, _I64, _P, _P, _D, _P, C.POINTER(cqk_spg_opts),
                                       C.POINTER(cqk_spg_info)]),
    "cqk_tune_batched_cqk_f64": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                           _P, C.c_int32, C.c_int32,
                                           C.POINTER(cqk_batch_schedule),
                                           C.POINTER(C.c_double)]),
    "cqk_tune_batched_cqk_f32": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                           _P, C.c_int32, C.c_int32,
                                           C.POINTER(cqk_batch_schedule),
                                           C.POINTER(C.c_double)]),
    "cqk_solve_warm_f64": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_solve_warm_f32": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_simplex_warm_f32": (C.c_int, [_P, _I64, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_simplex_warm_f64": (C.c_int, [_P, _I64, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_l1_warm_f32": (C.c_int, [_P, _I64, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_l1_warm_f64": (C.c_int, [_P, _I64, _P, _P, _D, _P, _OPTS, _INFO]),
    "cqk_project_simplex_batched_f32": (
        C.c_int, [_P, _I32, _P, _P, _P, _D, _P, _P, _P, _OPTS, _INFO]),
    "cqk_project_simplex_batched_noalloc_f32": (
        C.c_int, [_P, _I32, _P, _P, _P, _D, _P, _P, _P, _OPTS, _INFO]),
    "cqk_project_simplex_batched_backward_f32": (
        C.c_int, [_P, _I32, _P, _P, _P, _P, _P, _OPTS]),
    "cqk_get_compact_theta": (C.c_int, [_P, C.POINTER(_D)]),
    "cqk_set_compact_theta": (C.c_int, [_P, _D]),
    "cqk_tune_theta_f64": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _D, _P, _OPTS, _I32,
                                     C.POINTER(_D), C.POINTER(_D), _P]),
    "cqk_tune_theta_f32": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _D, _P, _OPTS, _I32,
                                     C.POINTER(_D), C.POINTER(_D), _P]),
    "cqk_get_batch_schedule": (C.c_int, [_P, _I32, C.POINTER(cqk_batch_schedule)]),
    "cqk_set_batch_schedule": (C.c_int, [_P, _I32, C.POINTER(cqk_batch_schedule)]),
    "cqk_tune_batched_f32": (
        C.c_int, [_P, _I32, _P, _P, _P, _D, _P, _I32, C.POINTER(cqk_batch_schedule),
                  C.POINTER(_D)]),
    "cqk_tune_batched_backward_f32": (
        C.c_int, [_P, _I32, _P, _P, _P, _P, _I32, C.POINTER(cqk_batch_schedule),
                  C.POINTER(_D)]),
}

_lib = None


def load(path: str | None = None):
    """Load libcqk.so once and declare its entry points."""
    global _lib
    if _lib is not None:
        return _lib
    # CQK_LIBRARY: another build of the same library (e.g. a tuning variant)
    p = path or os.environ.get("CQK_LIBRARY") or LIB_PATH
    if not os.path.exists(p):
        raise CqkLibraryMissing(
            f"{p} is not built; run `python -m paper_2603_15910_amd.build` "
            "(hipcc, gfx950). There is no CPU fallback.")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
