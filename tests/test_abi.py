"""Host-only checks of the C ABI: the library loads and exports every entry
point that include/cqk.h declares; the ctypes structs have the C layout;
host-side argument errors are reported without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2603_15910_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(cqk_[a-z0-9_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libcqk.so is not built (run __graft_entry__.build())")
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 15
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.SIGNATURES) == declared


def test_struct_layouts_match_header():
    # offsets follow from the C declarations with natural alignment
    assert C.sizeof(L.cqk_opts) == 64
    assert L.cqk_opts.lambda0_user.offset == 8
    assert L.cqk_opts.timing.offset == 60
    assert C.sizeof(L.cqk_info) == 112
    assert L.cqk_info.lambda_.offset == 16
    assert C.sizeof(L.cqk_trace_rec) == 72
    assert C.sizeof(L.cqk_batch_schedule) == 16


def test_status_strings_and_defaults(lib):
    assert lib.cqk_status_string(0) == b"CQK_OK"
    assert lib.cqk_status_string(1) == b"CQK_INFEASIBLE"
    assert lib.cqk_status_string(99) == b"CQK_UNKNOWN_STATUS"
    o = L.cqk_opts()
    lib.cqk_default_opts(C.byref(o))
    assert o.max_iter == 100 and o.compaction == 1 and o.sync == 1


def test_host_side_argument_errors(lib):
    # every case is rejected before a device is touched (null context)
    null = None
    assert lib.cqk_solve_f64(null, 10, null, null, null, null, null, 1.0, null, None, None) == 2
    assert lib.cqk_project_simplex_f32(null, 10, null, 1.0, null, None, None) == 2
    assert lib.cqk_project_l1_f64(null, 10, null, 1.0, null, None, None) == 2
    assert lib.cqk_solve_warm_f64(null, 10, null, null, null, null, null, null, 1.0, null, None,
                                  None) == 2
    assert lib.cqk_solve_warm_f32(null, 10, null, null, null, null, null, null, 1.0, null, None,
                                  None) == 2
    assert lib.cqk_project_simplex_warm_f32(null, 10, null, null, 1.0, null, None, None) == 2
    assert lib.cqk_project_simplex_warm_f64(null, 10, null, null, 1.0, null, None, None) == 2
    assert lib.cqk_project_l1_warm_f32(null, 10, null, null, 1.0, null, None, None) == 2
    assert lib.cqk_project_l1_warm_f64(null, 10, null, null, 1.0, null, None, None) == 2
    for name in ("cqk_project_simplex_sparse_f32", "cqk_project_simplex_sparse_f64",
                 "cqk_project_l1_sparse_f32", "cqk_project_l1_sparse_f64"):
        nnz = C.c_int64(-1)
        assert getattr(lib, name)(null, 10, null, null, 1.0, 4, null, null, C.byref(nnz), None,
                                  None) == 2
        assert nnz.value == 0
    assert lib.cqk_status_string(6) == b"CQK_BUFFER_TOO_SMALL"
    assert lib.cqk_spg_l1_lasso_f64(null, 4, 4, null, null, 1.0, null, None, None) == 2
    assert lib.cqk_solve_batched_f64(null, 2, null, null, null, null, null, null, null, null,
                                     null, null, None, None) == 2
    assert lib.cqk_solve_batched_backward_f64(null, 2, null, null, null, null, null, null, null,
                                              null, null, None) == 2
    assert lib.cqk_solve_batched_f32(null, 2, null, null, null, null, null, null, null, null,
                                     null, null, None, None) == 2
    assert lib.cqk_solve_batched_backward_f32(null, 2, null, null, null, null, null, null, null,
                                              null, null, None) == 2
    assert lib.cqk_tune_batched_cqk_f64(null, 4, null, null, null, null, null, null, null, null,
                                        null, null, 0, 3, None, None) == 2
    assert lib.cqk_tune_batched_cqk_f32(null, 4, null, null, null, null, null, null, null, null,
                                        null, null, 0, 3, None, None) == 2
    for which in (2, 3):
        assert lib.cqk_get_batch_schedule(null, which, C.byref(L.cqk_batch_schedule())) == 2
    so = L.cqk_spg_opts()
    lib.cqk_spg_default_opts(C.byref(so))
    assert so.tol == 1e-4 and so.max_iter == 10000 and so.memory == 10 and so.warm == 1
    assert lib.cqk_project_simplex_batched_f32(null, 4, null, null, null, 1.0, null, null, null,
                                               None, None) == 2
    assert lib.cqk_create(None, None) == 2
    assert lib.cqk_set_stream(null, null) == 2
    assert lib.cqk_last_trace(null, None, 0, None) == 2
    sc = L.cqk_batch_schedule(8, 4, 0, 0)
    assert lib.cqk_get_batch_schedule(null, 0, C.byref(sc)) == 2
    assert lib.cqk_set_batch_schedule(null, 0, C.byref(sc)) == 2
    assert lib.cqk_tune_batched_f32(null, 4, null, null, null, 1.0, null, 3, None, None) == 2
    assert lib.cqk_tune_batched_backward_f32(null, 4, null, null, null, null, 3, None,
                                             None) == 2
