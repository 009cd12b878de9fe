"""C-ABI checks that run without a GPU: the library loads, exports every
function that include/rid.h declares, and rejects bad calls before touching a
device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rid.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^RID_API [^;]*?\b(rid_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_documented_surface():
    names = declared_functions()
    for must in ("rid_context_create", "rid_problem_create", "rid_apply_operator", "rid_eigen_solve",
                 "rid_response_solve", "rid_batch_solve", "rid_server_submit", "rid_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2404_17133_amd import _binding as B

    lib = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding's prototype table covers the header exactly
    assert sorted(B.PROTOTYPES) == declared_functions()


def test_status_strings_and_defaults():
    from paper_2404_17133_amd import _binding as B

    assert B.lib.rid_status_string(0) == b"ok"
    assert b"not converged" in B.lib.rid_status_string(1)
    assert B.lib.rid_status_string(-6) == b"A-B not positive definite"
    o = B.rid_solve_opts()
    B.lib.rid_solve_opts_default(ctypes.byref(o))
    # defaults follow Sec. 3 and Sec. 3.1: 1e-5 outer, 1e-2 inner (<= 20), 1e-3 initial guess
    assert (o.tol, o.inner_tol, o.inner_max_iter, o.init_tol) == (1e-5, 1e-2, 20, 1e-3)
    assert o.n_extra_init == -1 and o.precond == B.RID_PRECOND_RIS


def test_null_arguments_rejected_without_device():
    from paper_2404_17133_amd import _binding as B

    L = B.lib
    assert L.rid_context_create(0, None, None, None) == B.RID_ERR_INVALID_ARG
    assert L.rid_context_destroy(None) == B.RID_ERR_INVALID_ARG
    assert L.rid_problem_destroy(None) == B.RID_ERR_INVALID_ARG
    assert L.rid_apply_operator(None, 0, 0, 1, None, None, None) == B.RID_ERR_INVALID_ARG
    assert L.rid_eigen_solve(None, None, 1, 0, None, None, None, None, None) == B.RID_ERR_INVALID_ARG
    assert L.rid_server_poll(None, 1) == B.RID_ERR_INVALID_ARG


def _dummy_allocator(B):
    fns = (B.ALLOC_FN(lambda user, n: None), B.FREE_FN(lambda user, p: None))
    return fns, B.rid_allocator(None, fns[0], fns[1])


def test_context_needs_an_allocator():
    """The library allocates device memory only through the caller's
    allocator: a missing allocator or callback is refused before any device
    is touched."""
    from paper_2404_17133_amd import _binding as B

    h = ctypes.c_void_p()
    assert B.lib.rid_context_create(0, None, None, ctypes.byref(h)) == B.RID_ERR_INVALID_ARG
    assert h.value is None
    assert b"allocator" in B.lib.rid_last_error(None)
    keep, al = _dummy_allocator(B)
    half = B.rid_allocator(None, keep[0], B.FREE_FN())
    assert B.lib.rid_context_create(0, None, ctypes.byref(half), ctypes.byref(h)) == B.RID_ERR_INVALID_ARG
    assert h.value is None


def test_context_without_gpu_reports_no_device():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2404_17133_amd import _binding as B

    keep, al = _dummy_allocator(B)
    h = ctypes.c_void_p()
    s = B.lib.rid_context_create(0, None, ctypes.byref(al), ctypes.byref(h))
    assert s == B.RID_ERR_NO_DEVICE
    assert h.value is None
    assert len(B.lib.rid_last_error(None)) > 0
