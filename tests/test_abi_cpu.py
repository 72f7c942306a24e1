"""The C-ABI library loads without a GPU, exports every function include/bccb.h
declares, and rejects bad arguments on the host before touching the device."""
import ctypes

import numpy as np
import pytest

B = pytest.importorskip("paper_2509_13592_amd.bccb")


def test_header_symbols_exported():
    names = B.declared_functions()
    # the calls of the boundary: plan, adjoint, Gram product, the three solvers, the
    # monitors, the batched solve and the learned network with its gated solve
    for n in ("bccb_plan", "bccb_plan_destroy", "bccb_plan_info", "bccb_adjoint", "bccb_gram_apply",
              "lasso_solve_ista", "lasso_solve_fista", "lasso_solve_admm", "lasso_solve_batch_fista",
              "bccb_kkt", "lista_forward", "lista_backward", "lista_solve", "bccb_status_string"):
        assert n in names, n
    for n in names:
        assert hasattr(B.lib, n), f"{n} declared in include/bccb.h but not exported"


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5):
        assert B.status_string(code).startswith("BCCB_")
    assert "unknown" in B.status_string(42)


def _plan(mask, M1, M2, L1, L2, out=True):
    h = ctypes.c_void_p()
    ptr = None if mask is None else mask.ctypes.data
    return B.lib.bccb_plan(ptr, M1, M2, L1, L2, None, ctypes.byref(h) if out else None)


@pytest.mark.parametrize("L1,L2,code", [(12, 16, -2), (16, 2048, -2), (4, 16, -2), (0, 16, -1), (16, -8, -1)])
def test_plan_rejects_grid_sizes(L1, L2, code):
    m = np.ones((4, 4), np.uint8)
    assert _plan(m, 4, 4, L1, L2) == code


def test_plan_rejects_bad_geometry():
    m = np.ones((4, 4), np.uint8)
    assert _plan(None, 4, 4, 16, 16) == B.BCCB_E_INVALID
    assert _plan(m, 0, 4, 16, 16) == B.BCCB_E_INVALID
    assert _plan(m, 4, 4, 16, 16, out=False) == B.BCCB_E_INVALID
    z = np.zeros((4, 4), np.uint8)
    assert _plan(z, 4, 4, 16, 16) == B.BCCB_E_INVALID       # empty array


def test_calls_reject_null_plan():
    d = ctypes.c_double()
    assert B.lib.lasso_solve_fista(None, None, 0.1, 10, None, None) == B.BCCB_E_INVALID
    assert B.lib.lasso_solve_ista(None, None, 0.1, 10, None, None) == B.BCCB_E_INVALID
    assert B.lib.lasso_solve_admm(None, None, 0.1, 1.0, 10, None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_gram_apply(None, None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_adjoint(None, None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_adjoint_maxabs(None, None, ctypes.byref(d)) == B.BCCB_E_INVALID
    assert B.lib.bccb_objective_kkt(None, None, 0.1, None, None, None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_plan_info(None, None, None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_kkt(None, None, 0.1, None, None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_plan_omega_device(None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_set_stream(None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_plan_destroy(None) == B.BCCB_OK
    assert B.lib.bccb_plan_support_columns(None, None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_plan_get_config(None, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_plan_autotune(None, 1, None) == B.BCCB_E_INVALID
    assert B.lib.bccb_batch_set_sparse_iterate(None, 1) == B.BCCB_E_INVALID
    assert B.lib.bccb_batch_set_support_columns(None, 1) == B.BCCB_E_INVALID
    assert B.lib.bccb_batch_class_config(None, 0, None) == B.BCCB_E_INVALID
    assert B.lib.lista_autotune(None, 1) == B.BCCB_E_INVALID
    assert B.lib.bccb_profile_resident(None, 1, 10, 1, ctypes.byref(d)) == B.BCCB_E_INVALID
    assert B.lib.bccb_stream_copy(None, None, ctypes.c_size_t(16), 0, None) == B.BCCB_E_INVALID
    # misaligned or ragged copies are refused before anything is enqueued
    assert B.lib.bccb_stream_copy(ctypes.c_void_p(16), ctypes.c_void_p(8), ctypes.c_size_t(16), 0, None) == \
        B.BCCB_E_INVALID
    assert B.lib.bccb_stream_copy(ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_size_t(24), 0, None) == \
        B.BCCB_E_INVALID
    assert B.lib.bccb_stream_copy(ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_size_t(16), 64, None) == \
        B.BCCB_E_INVALID


def test_binding_requires_gpu_tensors():
    import torch
    with pytest.raises((ValueError, TypeError)):
        B._ptr(torch.zeros(4, dtype=torch.complex64))
    with pytest.raises(TypeError):
        B._ptr(np.zeros(4))


def test_every_declared_function_has_a_signature():
    """The binding states argument types for every entry point of the header (a pointer
    or size passed without them would be truncated to a C int)."""
    missing = [name for name in B.declared_functions() if name not in B._SIGS]
    assert not missing, missing
