"""MI355X-native CQK / simplex / l1 projection library (HIP, gfx950).

The compute path lives in the HIP shared library ``libcqk.so`` (built from
``csrc/`` by ``paper_2603_15910_amd.build``).  This package is a thin binding
over its C ABI (``include/cqk.h``):

* the C entry points under their own names (``cqk_solve_f64`` ...), taking
  integer device pointers, exactly as declared in the header;
* ``Context`` and module-level helpers that take torch tensors on the GPU and
  pass ``data_ptr()`` and torch's current HIP stream;
* ``SimplexProjection``, a ``torch.autograd.Function`` whose forward and
  backward are the batched HIP kernels.

The library is loaded on first use; a missing build raises
``CqkLibraryMissing``.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import threading

from . import _lib as L
from ._lib import (CQK_BUFFER_TOO_SMALL, CQK_DEVICE_ERROR, CQK_INFEASIBLE, CQK_INVALID_ARG,
                   CQK_NO_MEMORY, CQK_NOALLOC_MAX_SEG, CQK_NOT_CONVERGED, CQK_OK, STATUS_NAMES,
                   CqkLibraryMissing, cqk_info, cqk_opts, cqk_trace_rec)

__all__ = [
    "CQK_OK", "CQK_INFEASIBLE", "CQK_INVALID_ARG", "CQK_NOT_CONVERGED", "CQK_DEVICE_ERROR",
    "CQK_NO_MEMORY", "CQK_BUFFER_TOO_SMALL", "CqkError", "CqkLibraryMissing", "Context", "solve",
    "project_simplex", "project_l1", "project_simplex_sparse", "project_l1_sparse",
    "solve_batched", "solve_batched_backward", "CqkBatchedSolve", "spg_l1_lasso",
    "project_simplex_batched", "project_simplex_batched_backward", "SimplexProjection", "lib",
]


def lib():
    return L.load()


class CqkError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}")


# ---------------------------------------------------------------------------
# The C entry points under their own names (pointer-level marshalling only)
# ---------------------------------------------------------------------------
def cqk_create(stream: int = 0) -> int:
    h = C.c_void_p()
    st = lib().cqk_create(C.byref(h), C.c_void_p(stream))
    if st != CQK_OK:
        raise CqkError(st, "cqk_create")
    return h.value


def cqk_destroy(ctx: int) -> None:
    lib().cqk_destroy(C.c_void_p(ctx))


def cqk_set_stream(ctx: int, stream: int) -> int:
    return lib().cqk_set_stream(C.c_void_p(ctx), C.c_void_p(stream))


def cqk_reserve(ctx: int, max_n: int, max_seg: int) -> int:
    return lib().cqk_reserve(C.c_void_p(ctx), max_n, max_seg)


def cqk_status_string(status: int) -> str:
    return lib().cqk_status_string(status).decode()


def cqk_default_opts() -> cqk_opts:
    o = cqk_opts()
    lib().cqk_default_opts(C.byref(o))
    return o


def cqk_last_trace(ctx: int, cap: int = 512):
    buf = (cqk_trace_rec * cap)()
    cnt = C.c_int32(0)
    lib().cqk_last_trace(C.c_void_p(ctx), buf, cap, C.byref(cnt))
    return [buf[i].as_dict() for i in range(min(cap, cnt.value))]


def cqk_last_pass_ms(ctx: int, cap: int = 1024):
    buf = (C.c_float * cap)()
    cnt = C.c_int32(0)
    lib().cqk_last_pass_ms(C.c_void_p(ctx), buf, cap, C.byref(cnt))
    return [float(buf[i]) for i in range(min(cap, cnt.value))]


def cqk_ctx_last_info(ctx: int):
    """(status, info dict) of the last call on the context, read from the
    device after waiting for its stream."""
    info = cqk_info()
    st = lib().cqk_ctx_last_info(C.c_void_p(ctx), C.byref(info))
    return st, info.as_dict()


def _call(name, *args):
    return getattr(lib(), name)(*args)


def cqk_solve_f64(ctx, n, d, a, b, l, u, r, x, opts=None, info=None):
    return _call("cqk_solve_f64", C.c_void_p(ctx), n, d, a, b, l, u, r, x,
                 C.byref(opts) if opts is not None else None,
                 C.byref(info) if info is not None else None)


def cqk_solve_f32(ctx, n, d, a, b, l, u, r, x, opts=None, info=None):
    return _call("cqk_solve_f32", C.c_void_p(ctx), n, d, a, b, l, u, r, x,
                 C.byref(opts) if opts is not None else None,
                 C.byref(info) if info is not None else None)


def _proj(name, ctx, n, y, r, x, opts, info):
    return _call(name, C.c_void_p(ctx), n, y, r, x,
                 C.byref(opts) if opts is not None else None,
                 C.byref(info) if info is not None else None)


def cqk_project_simplex_f32(ctx, n, y, r, x, opts=None, info=None):
    return _proj("cqk_project_simplex_f32", ctx, n, y, r, x, opts, info)


def cqk_project_simplex_f64(ctx, n, y, r, x, opts=None, info=None):
    return _proj("cqk_project_simplex_f64", ctx, n, y, r, x, opts, info)


def cqk_project_l1_f32(ctx, n, y, radius, x, opts=None, info=None):
    return _proj("cqk_project_l1_f32", ctx, n, y, radius, x, opts, info)


def cqk_project_l1_f64(ctx, n, y, radius, x, opts=None, info=None):
    return _proj("cqk_project_l1_f64", ctx, n, y, radius, x, opts, info)


def _ref(o):
    return C.byref(o) if o is not None else None


def cqk_solve_warm_f64(ctx, n, d, a, b, l, u, xbar, r, x, opts=None, info=None):
    return _call("cqk_solve_warm_f64", C.c_void_p(ctx), n, d, a, b, l, u, xbar, r, x,
                 _ref(opts), _ref(info))


def cqk_solve_warm_f32(ctx, n, d, a, b, l, u, xbar, r, x, opts=None, info=None):
    return _call("cqk_solve_warm_f32", C.c_void_p(ctx), n, d, a, b, l, u, xbar, r, x,
                 _ref(opts), _ref(info))


def cqk_project_simplex_warm_f32(ctx, n, y, xbar, r, x, opts=None, info=None):
    return _call("cqk_project_simplex_warm_f32", C.c_void_p(ctx), n, y, xbar, r, x,
                 _ref(opts), _ref(info))


def cqk_project_simplex_warm_f64(ctx, n, y, xbar, r, x, opts=None, info=None):
    return _call("cqk_project_simplex_warm_f64", C.c_void_p(ctx), n, y, xbar, r, x,
                 _ref(opts), _ref(info))


def cqk_project_l1_warm_f32(ctx, n, y, xbar, radius, x, opts=None, info=None):
    return _call("cqk_project_l1_warm_f32", C.c_void_p(ctx), n, y, xbar, radius, x,
                 _ref(opts), _ref(info))


def cqk_project_l1_warm_f64(ctx, n, y, xbar, radius, x, opts=None, info=None):
    return _call("cqk_project_l1_warm_f64", C.c_void_p(ctx), n, y, xbar, radius, x,
                 _ref(opts), _ref(info))


def _sparse(name, ctx, n, y, xbar, r, cap, idx, val, opts, info):
    nnz = C.c_int64(0)
    st = _call(name, C.c_void_p(ctx), n, y, xbar, r, cap, idx, val, C.byref(nnz), _ref(opts),
               _ref(info))
    return st, nnz.value


def cqk_project_simplex_sparse_f32(ctx, n, y, xbar, r, cap, idx, val, opts=None, info=None):
    """Returns (status, nnz)."""
    return _sparse("cqk_project_simplex_sparse_f32", ctx, n, y, xbar, r, cap, idx, val, opts, info)


def cqk_project_simplex_sparse_f64(ctx, n, y, xbar, r, cap, idx, val, opts=None, info=None):
    """Returns (status, nnz)."""
    return _sparse("cqk_project_simplex_sparse_f64", ctx, n, y, xbar, r, cap, idx, val, opts, info)


def cqk_project_l1_sparse_f32(ctx, n, y, xbar, radius, cap, idx, val, opts=None, info=None):
    """Returns (status, nnz)."""
    return _sparse("cqk_project_l1_sparse_f32", ctx, n, y, xbar, radius, cap, idx, val, opts,
                   info)


def cqk_project_l1_sparse_f64(ctx, n, y, xbar, radius, cap, idx, val, opts=None, info=None):
    """Returns (status, nnz)."""
    return _sparse("cqk_project_l1_sparse_f64", ctx, n, y, xbar, radius, cap, idx, val, opts,
                   info)


def cqk_spg_l1_lasso_f64(ctx, m, n, A, b, radius, x, opts=None, info=None):
    return _call("cqk_spg_l1_lasso_f64", C.c_void_p(ctx), m, n, A, b, radius, x, _ref(opts),
                 _ref(info))


def spg_opts(tol=1e-4, max_iter=10000, memory=10, warm=True):
    o = L.cqk_spg_opts()
    lib().cqk_spg_default_opts(C.byref(o))
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.memory = int(memory)
    o.warm = 1 if warm else 0
    return o


def cqk_solve_batched_f64(ctx, nseg, offsets, d, a, b, l, u, r, x, lambda_out=None,
                          status_out=None, opts=None, info=None):
    return _call("cqk_solve_batched_f64", C.c_void_p(ctx), nseg, offsets, d, a, b, l, u, r, x,
                 lambda_out, status_out, _ref(opts), _ref(info))


def cqk_solve_batched_backward_f64(ctx, nseg, offsets, x, g, d, b, l, u, grad_a, grad_r=None,
                                   opts=None):
    return _call("cqk_solve_batched_backward_f64", C.c_void_p(ctx), nseg, offsets, x, g, d, b,
                 l, u, grad_a, grad_r, _ref(opts))


def cqk_solve_batched_f32(ctx, nseg, offsets, d, a, b, l, u, r, x, lambda_out=None,
                          status_out=None, opts=None, info=None):
    return _call("cqk_solve_batched_f32", C.c_void_p(ctx), nseg, offsets, d, a, b, l, u, r, x,
                 lambda_out, status_out, _ref(opts), _ref(info))


def cqk_solve_batched_backward_f32(ctx, nseg, offsets, x, g, d, b, l, u, grad_a, grad_r=None,
                                   opts=None):
    return _call("cqk_solve_batched_backward_f32", C.c_void_p(ctx), nseg, offsets, x, g, d, b,
                 l, u, grad_a, grad_r, _ref(opts))


def cqk_project_simplex_batched_f32(ctx, nseg, offsets, y, r, r_scalar, x, lambda_out=None,
                                    nfree_out=None, opts=None, info=None):
    return _call("cqk_project_simplex_batched_f32", C.c_void_p(ctx), nseg, offsets, y, r,
                 r_scalar, x, lambda_out, nfree_out,
                 C.byref(opts) if opts is not None else None,
                 C.byref(info) if info is not None else None)


def cqk_project_simplex_batched_noalloc_f32(ctx, nseg, offsets, y, r, r_scalar, x,
                                            lambda_out=None, nfree_out=None, opts=None,
                                            info=None):
    return _call("cqk_project_simplex_batched_noalloc_f32", C.c_void_p(ctx), nseg, offsets, y,
                 r, r_scalar, x, lambda_out, nfree_out,
                 C.byref(opts) if opts is not None else None,
                 C.byref(info) if info is not None else None)


def cqk_project_simplex_batched_backward_f32(ctx, nseg, offsets, x, g, grad_y, grad_r=None,
                                             opts=None):
    return _call("cqk_project_simplex_batched_backward_f32", C.c_void_p(ctx), nseg, offsets, x,
                 g, grad_y, grad_r, C.byref(opts) if opts is not None else None)


def cqk_get_batch_schedule(ctx, backward=0):
    sc = L.cqk_batch_schedule()
    st = _call("cqk_get_batch_schedule", C.c_void_p(ctx), int(backward), C.byref(sc))
    return st, sc


def cqk_set_batch_schedule(ctx, backward, sched):
    return _call("cqk_set_batch_schedule", C.c_void_p(ctx), int(backward), C.byref(sched))


def cqk_tune_batched_f32(ctx, nseg, offsets, y, r, r_scalar, x, repeats=3):
    sc = L.cqk_batch_schedule()
    ms = C.c_double(0.0)
    st = _call("cqk_tune_batched_f32", C.c_void_p(ctx), nseg, offsets, y, r, r_scalar, x,
               int(repeats), C.byref(sc), C.byref(ms))
    return st, sc, ms.value


def cqk_tune_batched_backward_f32(ctx, nseg, offsets, x, g, grad_y, repeats=3):
    sc = L.cqk_batch_schedule()
    ms = C.c_double(0.0)
    st = _call("cqk_tune_batched_backward_f32", C.c_void_p(ctx), nseg, offsets, x, g, grad_y,
               int(repeats), C.byref(sc), C.byref(ms))
    return st, sc, ms.value


# ---------------------------------------------------------------------------
# torch-tensor helpers
# ---------------------------------------------------------------------------
def make_opts(lambda0=None, lambda0_user=0.0, max_iter=100, tol=0.0, compaction="auto",
              theta=0.0, accum="default", trace=False, timing=False, simplex=False, sync=True):
    o = cqk_default_opts()
    if lambda0 is None:
        lambda0 = "condat" if simplex else "zero"
    o.lambda0_mode = L.LAMBDA0[lambda0]
    o.lambda0_user = float(lambda0_user)
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.compaction = L.COMPACTION[compaction]
    o.compact_theta = float(theta)
    o.accum = L.ACCUM[accum]
    o.sync = 1 if sync else 0
    o.trace = 1 if trace else 0
    # True: every pass kernel; 2: the first Newton pass and the x-writing pass
    o.timing = int(timing) if not isinstance(timing, bool) else (1 if timing else 0)
    return o


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


class Context:
    """One libcqk context (workspace + state) on one GPU."""

    def __init__(self, device=None):
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.handle = cqk_create(torch.cuda.current_stream(self.device).cuda_stream)
        self.last_info = None

    def close(self):
        if self.handle:
            cqk_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self):
        torch = _torch()
        cqk_set_stream(self.handle, torch.cuda.current_stream(self.device).cuda_stream)

    def reserve(self, max_n, max_seg=0):
        st = cqk_reserve(self.handle, int(max_n), int(max_seg))
        if st != CQK_OK:
            raise CqkError(st, "cqk_reserve")

    def trace(self):
        return cqk_last_trace(self.handle)

    def pass_ms(self):
        """Kernel ms of each grid pass of the last timed single-instance call."""
        return cqk_last_pass_ms(self.handle)

    def ctx_last_info(self):
        """(status, info) of the last call, read from the device: the outcome
        of a call made with sync=False or replayed from a captured graph.
        Waits for torch's current stream (where a replay was launched)."""
        self._bind_stream()
        return cqk_ctx_last_info(self.handle)

    def solve(self, d, a, b, l, u, r, out=None, check=True, xbar=None, **kw):
        """General CQK.  xbar: a primal estimate (same dtype and size) for
        the warm start; lambda0 options are then ignored."""
        torch = _torch()
        dt = d.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("solve takes float64 or float32 tensors")
        n = d.numel()
        x = out if out is not None else torch.empty_like(d)
        ptrs = [_dev_ptr(t, dt, nm) for t, nm in zip((d, a, b, l, u, x), "dablux")]
        opts = make_opts(**kw)
        info = cqk_info()
        self._bind_stream()
        if xbar is None:
            fn = cqk_solve_f64 if dt == torch.float64 else cqk_solve_f32
            st = fn(self.handle, n, *ptrs[:5], float(r), ptrs[5], opts, info)
        else:
            pw = _dev_ptr(xbar, dt, "xbar")
            if xbar.numel() != n:
                raise ValueError("xbar must have as many elements as d")
            fn = cqk_solve_warm_f64 if dt == torch.float64 else cqk_solve_warm_f32
            st = fn(self.handle, n, *ptrs[:5], pw, float(r), ptrs[5], opts, info)
        self.last_info = info.as_dict()
        if check and st not in (CQK_OK,):
            raise CqkError(st, "cqk_solve")
        return x, self.last_info

    def _project(self, name64, name32, y, r, out, check, kw, xbar=None, warm=None):
        torch = _torch()
        x = out if out is not None else torch.empty_like(y)
        dt = y.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("projection takes float64 or float32 tensors")
        py = _dev_ptr(y, dt, "y")
        px = _dev_ptr(x, dt, "x")
        opts = make_opts(simplex=True, **kw)
        info = cqk_info()
        self._bind_stream()
        if xbar is None:
            fn = name64 if dt == torch.float64 else name32
            st = fn(self.handle, y.numel(), py, float(r), px, opts, info)
        else:
            pw = _dev_ptr(xbar, dt, "xbar")
            if xbar.numel() != y.numel():
                raise ValueError("xbar must have as many elements as y")
            fn = warm[0] if dt == torch.float64 else warm[1]
            st = fn(self.handle, y.numel(), py, pw, float(r), px, opts, info)
        self.last_info = info.as_dict()
        if check and st != CQK_OK:
            raise CqkError(st, fn.__name__)
        return x, self.last_info

    def project_simplex(self, y, r=1.0, out=None, check=True, xbar=None, **kw):
        """Projection onto the r-simplex.  xbar: a primal estimate for the
        warm start (Algorithm 2 over its support)."""
        return self._project(cqk_project_simplex_f64, cqk_project_simplex_f32, y, r, out, check,
                             kw, xbar, (cqk_project_simplex_warm_f64, cqk_project_simplex_warm_f32))

    def project_l1(self, y, radius=1.0, out=None, check=True, xbar=None, **kw):
        """Projection onto the l1 ball.  xbar: a primal estimate for the warm
        start (Algorithm 2 over {xbar != 0})."""
        return self._project(cqk_project_l1_f64, cqk_project_l1_f32, y, radius, out, check, kw,
                             xbar, (cqk_project_l1_warm_f64, cqk_project_l1_warm_f32))

    def _project_sparse(self, names, y, r, cap, xbar, check, kw, out=None):
        torch = _torch()
        dt = y.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("projection takes float64 or float32 tensors")
        n = y.numel()
        py = _dev_ptr(y, dt, "y")
        pw = None
        if xbar is not None:
            pw = _dev_ptr(xbar, dt, "xbar")
            if xbar.numel() != n:
                raise ValueError("xbar must have as many elements as y")
        fn = names[0] if dt == torch.float64 else names[1]
        opts = make_opts(simplex=True, **kw)
        info = cqk_info()
        self._bind_stream()
        if out is not None:
            idx, val = out
            _dev_ptr(idx, torch.int64, "out[0]")
            _dev_ptr(val, dt, "out[1]")
            cap = min(idx.numel(), val.numel())
        else:
            cap = min(n, 1 << 16) if cap is None else int(cap)
        for attempt in range(2):
            if out is None or attempt == 1:
                idx = torch.empty(max(cap, 1), dtype=torch.int64, device=y.device)
                val = torch.empty(max(cap, 1), dtype=dt, device=y.device)
            st, nnz = fn(self.handle, n, py, pw, float(r), cap, idx.data_ptr(), val.data_ptr(),
                         opts, info)
            if st != CQK_BUFFER_TOO_SMALL or attempt == 1:
                break
            cap = nnz   # the support is known now: solve once more into room for it
        self.last_info = info.as_dict()
        self.last_info["nnz"] = nnz
        if check and st != CQK_OK:
            raise CqkError(st, fn.__name__)
        return idx[:nnz], val[:nnz], self.last_info

    def project_simplex_sparse(self, y, r=1.0, cap=None, xbar=None, check=True, out=None, **kw):
        """Projection onto the r-simplex returned as its support: (indices
        ascending, int64; values; info).  cap: room for the support (default
        min(n, 65536); a larger support is solved once more with room for
        it).  out: (int64 tensor, value tensor) to write into instead, the
        room being their size.  xbar: a warm-start estimate."""
        return self._project_sparse((cqk_project_simplex_sparse_f64,
                                     cqk_project_simplex_sparse_f32), y, r, cap, xbar, check, kw,
                                    out)

    def project_l1_sparse(self, y, radius=1.0, cap=None, xbar=None, check=True, out=None, **kw):
        """Projection onto the l1 ball returned as its support (see
        project_simplex_sparse)."""
        return self._project_sparse((cqk_project_l1_sparse_f64, cqk_project_l1_sparse_f32), y,
                                    radius, cap, xbar, check, kw, out)

    def solve_batched(self, d, a, b, l, u, offsets, r, out=None, lambda_out=None,
                      status_out=None, check=True, **kw):
        """Many general CQK rows in one launch: row s is [offsets[s],
        offsets[s+1]) of the arrays d, a, b, l, u (all float64, or all
        float32 with float64 arithmetic); r a float64 GPU tensor [nseg].
        Returns (x, info)."""
        torch = _torch()
        nseg = offsets.numel() - 1
        dt = d.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("solve_batched takes float64 or float32 arrays")
        fn = cqk_solve_batched_f64 if dt == torch.float64 else cqk_solve_batched_f32
        x = out if out is not None else torch.empty_like(d)
        ptrs = [_dev_ptr(t, dt, nm) for t, nm in zip((d, a, b, l, u, x), "dablux")]
        po = _dev_ptr(offsets, torch.int64, "offsets")
        pr = _dev_ptr(r, torch.float64, "r")
        if r.numel() != nseg:
            raise ValueError("r needs one value per row")
        pl = _dev_ptr(lambda_out, torch.float64, "lambda_out") if lambda_out is not None else None
        ps = _dev_ptr(status_out, torch.int32, "status_out") if status_out is not None else None
        opts = make_opts(**kw)
        info = cqk_info()
        self._bind_stream()
        st = fn(self.handle, nseg, po, *ptrs[:5], pr, ptrs[5], pl, ps, opts, info)
        self.last_info = info.as_dict()
        if check and st != CQK_OK:
            raise CqkError(st, fn.__name__)
        return x, self.last_info

    def solve_batched_backward(self, x, g, d, b, l, u, offsets, grad_a=None, grad_r=None,
                               check=True, **kw):
        """VJP of solve_batched w.r.t. a (returned) and r (into grad_r)."""
        torch = _torch()
        nseg = offsets.numel() - 1
        dt = d.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("solve_batched_backward takes float64 or float32 arrays")
        fn = (cqk_solve_batched_backward_f64 if dt == torch.float64
              else cqk_solve_batched_backward_f32)
        ga = grad_a if grad_a is not None else torch.empty_like(g)
        ptrs = [_dev_ptr(t, dt, nm)
                for t, nm in zip((x, g, d, b, l, u, ga), ("x", "g", "d", "b", "l", "u", "grad_a"))]
        po = _dev_ptr(offsets, torch.int64, "offsets")
        pgr = _dev_ptr(grad_r, torch.float64, "grad_r") if grad_r is not None else None
        opts = make_opts(**kw)
        self._bind_stream()
        st = fn(self.handle, nseg, po, *ptrs, pgr, opts)
        if check and st != CQK_OK:
            raise CqkError(st, fn.__name__)
        return ga

    def spg_l1_lasso(self, A, b, radius, out=None, check=True, **kw):
        """min 1/2||A x - b||^2 s.t. ||x||_1 <= radius by SPG with warm-started
        l1 projections.  A: float64 GPU tensor [m, n] (row-major), b [m].
        kw: tol, max_iter, memory, warm.  Returns (x, info)."""
        torch = _torch()
        if A.dim() != 2:
            raise ValueError("A must be a matrix")
        m, n = A.shape
        if b.numel() != m:
            raise ValueError("b needs one value per row of A")
        x = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
        pa = _dev_ptr(A, torch.float64, "A")
        pb = _dev_ptr(b, torch.float64, "b")
        px = _dev_ptr(x, torch.float64, "x")
        info = L.cqk_spg_info()
        self._bind_stream()
        st = cqk_spg_l1_lasso_f64(self.handle, m, n, pa, pb, float(radius), px, spg_opts(**kw),
                                  info)
        self.last_info = info.as_dict()
        if check and st != CQK_OK:
            raise CqkError(st, "cqk_spg_l1_lasso_f64")
        return x, self.last_info

    def project_simplex_batched(self, y, offsets, r=1.0, out=None, lambda_out=None,
                                nfree_out=None, check=True, noalloc=False, **kw):
        """Batched simplex projection of the rows y[offsets[s]:offsets[s+1]].
        noalloc=True calls cqk_project_simplex_batched_noalloc_f32 (fixed
        planning buffers, no device allocation, at most CQK_NOALLOC_MAX_SEG
        rows)."""
        torch = _torch()
        nseg = offsets.numel() - 1
        x = out if out is not None else torch.empty_like(y)
        py = _dev_ptr(y, torch.float32, "y")
        px = _dev_ptr(x, torch.float32, "x")
        po = _dev_ptr(offsets, torch.int64, "offsets")
        if torch.is_tensor(r):
            pr, rs = _dev_ptr(r, torch.float64, "r"), 0.0
        else:
            pr, rs = None, float(r)
        pl = _dev_ptr(lambda_out, torch.float64, "lambda_out") if lambda_out is not None else None
        pn = _dev_ptr(nfree_out, torch.int32, "nfree_out") if nfree_out is not None else None
        opts = make_opts(simplex=True, **kw)
        info = cqk_info()
        self._bind_stream()
        fn = (cqk_project_simplex_batched_noalloc_f32 if noalloc
              else cqk_project_simplex_batched_f32)
        st = fn(self.handle, nseg, po, py, pr, rs, px, pl, pn, opts, info)
        self.last_info = info.as_dict()
        if check and st != CQK_OK:
            raise CqkError(st, fn.__name__)
        return x, self.last_info

    def project_simplex_batched_backward(self, x, g, offsets, grad_y=None, grad_r=None,
                                         check=True, **kw):
        torch = _torch()
        nseg = offsets.numel() - 1
        gy = grad_y if grad_y is not None else torch.empty_like(g)
        px = _dev_ptr(x, torch.float32, "x")
        pg = _dev_ptr(g, torch.float32, "g")
        pgy = _dev_ptr(gy, torch.float32, "grad_y")
        po = _dev_ptr(offsets, torch.int64, "offsets")
        pgr = _dev_ptr(grad_r, torch.float64, "grad_r") if grad_r is not None else None
        opts = make_opts(simplex=True, **kw)
        self._bind_stream()
        st = cqk_project_simplex_batched_backward_f32(self.handle, nseg, po, px, pg, pgy, pgr,
                                                      opts)
        if check and st != CQK_OK:
            raise CqkError(st, "cqk_project_simplex_batched_backward_f32")
        return gy


    @property
    def compact_theta(self):
        """The compaction threshold AUTO solves use when they give none."""
        v = C.c_double(0.0)
        st = _call("cqk_get_compact_theta", C.c_void_p(self.handle), C.byref(v))
        if st != CQK_OK:
            raise CqkError(st, "cqk_get_compact_theta")
        return v.value

    @compact_theta.setter
    def compact_theta(self, theta):
        st = _call("cqk_set_compact_theta", C.c_void_p(self.handle), float(theta))
        if st != CQK_OK:
            raise CqkError(st, "cqk_set_compact_theta")

    def tune_theta(self, d, a, b, l, u, r, repeats=3, out=None, **kw):
        """Times the general solve of this instance at every candidate
        theta (L.THETA_CANDIDATES) and keeps the fastest as the context's;
        returns (theta, ms, {theta: ms}).  kw: solve options (compaction is
        AUTO)."""
        torch = _torch()
        dt = d.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("tune_theta takes float64 or float32 tensors")
        n = d.numel()
        x = out if out is not None else torch.empty_like(d)
        ptrs = [_dev_ptr(t, dt, nm) for t, nm in zip((d, a, b, l, u, x), "dablux")]
        opts = make_opts(**kw)
        best, ms = C.c_double(0.0), C.c_double(0.0)
        times = (C.c_double * L.CQK_THETA_CANDIDATES)()
        name = "cqk_tune_theta_f64" if dt == torch.float64 else "cqk_tune_theta_f32"
        self._bind_stream()
        st = _call(name, C.c_void_p(self.handle), n, *ptrs[:5], float(r), ptrs[5],
                   C.byref(opts), int(repeats), C.byref(best), C.byref(ms),
                   C.cast(times, C.c_void_p))
        if st != CQK_OK:
            raise CqkError(st, name)
        return best.value, ms.value, dict(zip(L.THETA_CANDIDATES, list(times)))

    def batch_schedule(self, backward=False, general=False):
        """The context's batched schedule as a dict (general: the batched
        general CQK's, else the batched simplex's)."""
        st, sc = cqk_get_batch_schedule(self.handle, (2 if general else 0) + (1 if backward else 0))
        if st != CQK_OK:
            raise CqkError(st, "cqk_get_batch_schedule")
        return sc.as_dict()

    def set_batch_schedule(self, small_per=8, blocks_per_cu=4, short_first=0, backward=False,
                           general=False, medium_tiles=0):
        sc = L.cqk_batch_schedule(int(small_per), int(blocks_per_cu), int(short_first),
                                  int(medium_tiles))
        st = cqk_set_batch_schedule(self.handle, (2 if general else 0) + (1 if backward else 0),
                                    sc)
        if st != CQK_OK:
            raise CqkError(st, "cqk_set_batch_schedule")

    def tune_batched_cqk(self, d, a, b, l, u, offsets, r, repeats=3, backward=False, x=None,
                         g=None):
        """Times every candidate schedule of the batched general CQK forward
        (or, backward=True, of its VJP: needs x and g) on these rows and keeps
        the fastest in the context; returns (schedule dict, ms).  The arrays
        are all float64 or all float32 (r float64), as for solve_batched."""
        torch = _torch()
        nseg = offsets.numel() - 1
        dt = d.dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("tune_batched_cqk takes float64 or float32 arrays")
        name = "cqk_tune_batched_cqk_f64" if dt == torch.float64 else "cqk_tune_batched_cqk_f32"
        xx = x if x is not None else torch.empty_like(d)
        ga = torch.empty_like(d) if backward else None
        ptr = lambda t, nm: _dev_ptr(t, dt, nm) if t is not None else None
        sc = L.cqk_batch_schedule()
        ms = C.c_double(0.0)
        self._bind_stream()
        st = _call(name, C.c_void_p(self.handle), nseg,
                   _dev_ptr(offsets, torch.int64, "offsets"), ptr(d, "d"), ptr(a, "a"),
                   ptr(b, "b"), ptr(l, "l"), ptr(u, "u"),
                   _dev_ptr(r, torch.float64, "r") if r is not None else None, ptr(xx, "x"),
                   ptr(g, "g"), ptr(ga, "grad_a"), 1 if backward else 0, int(repeats),
                   C.byref(sc), C.byref(ms))
        if st != CQK_OK:
            raise CqkError(st, name)
        return sc.as_dict(), ms.value

    def tune_batched(self, y, offsets, r=1.0, repeats=3, out=None):
        """Times every candidate schedule on these rows and keeps the fastest
        for later batched forward calls; returns (schedule dict, ms)."""
        torch = _torch()
        nseg = offsets.numel() - 1
        x = out if out is not None else torch.empty_like(y)
        py = _dev_ptr(y, torch.float32, "y")
        px = _dev_ptr(x, torch.float32, "x")
        po = _dev_ptr(offsets, torch.int64, "offsets")
        if torch.is_tensor(r):
            pr, rs = _dev_ptr(r, torch.float64, "r"), 0.0
        else:
            pr, rs = None, float(r)
        self._bind_stream()
        st, sc, ms = cqk_tune_batched_f32(self.handle, nseg, po, py, pr, rs, px, repeats)
        if st != CQK_OK:
            raise CqkError(st, "cqk_tune_batched_f32")
        return sc.as_dict(), ms

    def tune_batched_backward(self, x, g, offsets, repeats=3, grad_y=None):
        """The same for the backward call; returns (schedule dict, ms)."""
        torch = _torch()
        nseg = offsets.numel() - 1
        gy = grad_y if grad_y is not None else torch.empty_like(g)
        px = _dev_ptr(x, torch.float32, "x")
        pg = _dev_ptr(g, torch.float32, "g")
        pgy = _dev_ptr(gy, torch.float32, "grad_y")
        po = _dev_ptr(offsets, torch.int64, "offsets")
        self._bind_stream()
        st, sc, ms = cqk_tune_batched_backward_f32(self.handle, nseg, po, px, pg, pgy, repeats)
        if st != CQK_OK:
            raise CqkError(st, "cqk_tune_batched_backward_f32")
        return sc.as_dict(), ms


_ctx_lock = threading.Lock()
_contexts = {}


def default_context(device=None) -> Context:
    torch = _torch()
    idx = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    key = (threading.get_ident(), idx)
    with _ctx_lock:
        if key not in _contexts:
            _contexts[key] = Context(idx)
        return _contexts[key]


def solve(d, a, b, l, u, r, **kw):
    return default_context(d.device).solve(d, a, b, l, u, r, **kw)


def project_simplex(y, r=1.0, **kw):
    return default_context(y.device).project_simplex(y, r, **kw)


def project_l1(y, radius=1.0, **kw):
    return default_context(y.device).project_l1(y, radius, **kw)


def project_simplex_sparse(y, r=1.0, **kw):
    return default_context(y.device).project_simplex_sparse(y, r, **kw)


def project_l1_sparse(y, radius=1.0, **kw):
    return default_context(y.device).project_l1_sparse(y, radius, **kw)


def project_simplex_batched(y, offsets, r=1.0, **kw):
    return default_context(y.device).project_simplex_batched(y, offsets, r, **kw)


def project_simplex_batched_backward(x, g, offsets, **kw):
    return default_context(x.device).project_simplex_batched_backward(x, g, offsets, **kw)


def spg_l1_lasso(A, b, radius, **kw):
    return default_context(A.device).spg_l1_lasso(A, b, radius, **kw)


def solve_batched(d, a, b, l, u, offsets, r, **kw):
    return default_context(d.device).solve_batched(d, a, b, l, u, offsets, r, **kw)


def solve_batched_backward(x, g, d, b, l, u, offsets, **kw):
    return default_context(x.device).solve_batched_backward(x, g, d, b, l, u, offsets, **kw)


def _autograd_cls():
    torch = _torch()

    class _SimplexProjection(torch.autograd.Function):
        """Batched simplex projection with a hand-written HIP backward.

        forward(y, offsets, r): y float32 [N], offsets int64 [nseg+1] (GPU),
        r a float or a float64 GPU tensor [nseg].  backward returns
        (grad_y, None, grad_r): grad_r per row when r is a tensor, None when
        r is a Python number (not a graph input, so autograd takes no
        gradient for it)."""

        @staticmethod
        def forward(ctx, y, offsets, r):
            x, _ = project_simplex_batched(y.contiguous(), offsets, r)
            ctx.save_for_backward(x, offsets)
            ctx.r_is_tensor = torch.is_tensor(r)
            return x

        @staticmethod
        def backward(ctx, g):
            x, offsets = ctx.saved_tensors
            nseg = offsets.numel() - 1
            grad_r = torch.empty(nseg, dtype=torch.float64, device=x.device)
            gy = project_simplex_batched_backward(x, g.contiguous().float(), offsets,
                                                  grad_r=grad_r)
            gr = grad_r if ctx.r_is_tensor else None
            return gy, None, gr

    class _CqkBatchedSolve(torch.autograd.Function):
        """Batched general CQK with a hand-written HIP backward.

        forward(d, a, b, l, u, offsets, r): float64 (or all float32) GPU
        tensors, offsets int64 [nseg+1], r float64 [nseg].  Differentiable in a and r;
        backward returns (None, grad_a, None, None, None, None, grad_r)."""

        @staticmethod
        def forward(ctx, d, a, b, l, u, offsets, r):
            x, _ = solve_batched(d, a.contiguous(), b, l, u, offsets, r)
            ctx.save_for_backward(x, d, b, l, u, offsets)
            return x

        @staticmethod
        def backward(ctx, g):
            x, d, b, l, u, offsets = ctx.saved_tensors
            nseg = offsets.numel() - 1
            grad_r = torch.empty(nseg, dtype=torch.float64, device=x.device)
            ga = solve_batched_backward(x, g.contiguous().to(x.dtype), d, b, l, u, offsets,
                                        grad_r=grad_r)
            return None, ga, None, None, None, None, grad_r

    return _SimplexProjection, _CqkBatchedSolve


class _Lazy:
    _cls = None

    def __init__(self, which):
        self._which = which

    def __getattr__(self, item):
        if _Lazy._cls is None:
            _Lazy._cls = _autograd_cls()
        return getattr(_Lazy._cls[self._which], item)


SimplexProjection = _Lazy(0)
CqkBatchedSolve = _Lazy(1)
