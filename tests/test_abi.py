"""The C-ABI library loads and exports every function include/setd.h declares;
host-side argument validation works without a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_2310_07551_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "setd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(setd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("setd_phi_matrices", "setd_tucker_apply", "setd_split_phi_apply", "setd_etd_step",
                     "setd_ctx_create", "setd_ctx_destroy", "setd_last_error", "setd_sync"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES), "binding signatures out of sync with the header"


def test_version_and_empty_error():
    lib = _lib.load()
    assert b"gfx950" in lib.setd_version()
    assert lib.setd_last_error() is not None


def test_workspace_size_is_host_only():
    lib = _lib.load()
    dims = (ctypes.c_int64 * 3)(256, 256, 256)
    nbytes = lib.setd_tucker_workspace_bytes(3, dims, _lib.PREC_F64)
    assert nbytes >= 2 * 256 ** 3 * 8
    assert lib.setd_tucker_workspace_bytes(0, dims, _lib.PREC_F64) == 0
    bad = (ctypes.c_int64 * 3)(256, 0, 256)
    assert lib.setd_tucker_workspace_bytes(3, bad, _lib.PREC_F64) == 0
    # more than 2^36 elements: rejected before any size product can overflow
    huge = (ctypes.c_int64 * 8)(*([4096] * 8))
    assert lib.setd_tucker_workspace_bytes(8, huge, _lib.PREC_F64) == 0
    edge = (ctypes.c_int64 * 3)(4096, 4096, 4096)          # exactly 2^36
    assert lib.setd_tucker_workspace_bytes(3, edge, _lib.PREC_F64) > 2 ** 36 * 8


def test_validation_errors_before_any_launch():
    lib = _lib.load()
    assert lib.setd_phi_matrices(None, 4, 0.1, 1, None, None) == _lib.SETD_EINVAL
    assert b"non-NULL" in lib.setd_last_error()
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 3)(8, 8, 8)
    A = (ctypes.c_void_p * 6)()
    assert lib.setd_ctx_create(ctypes.byref(h), 4, dims, 2, A, 0.01, 0, None) == _lib.SETD_EINVAL
    assert lib.setd_ctx_create(ctypes.byref(h), 3, dims, 3, A, 0.01, 0, None) == _lib.SETD_EINVAL
    assert lib.setd_ctx_create(ctypes.byref(h), 3, dims, 2, A, -1.0, 0, None) == _lib.SETD_EINVAL
    assert lib.setd_ctx_create(ctypes.byref(h), 3, dims, 2, A, 0.01, 0, None) == _lib.SETD_EINVAL   # NULL A
    assert lib.setd_split_phi_apply(None, 0, 1, 2, None, None, 1.0, 0.0, None) == _lib.SETD_EINVAL
    p = (ctypes.c_double * 1)(0.0)
    assert lib.setd_etd_step(None, None, 1, 0.01, 0, p, 0, None) == _lib.SETD_EINVAL
    dd = (ctypes.c_int64 * 2)(4, 4)
    M = (ctypes.c_void_p * 2)()
    assert lib.setd_tucker_apply(None, None, 2, dd, M, 1.0, 0.0, 0, None, 0, None) == _lib.SETD_EINVAL
    huge = (ctypes.c_int64 * 8)(*([4096] * 8))
    M8 = (ctypes.c_void_p * 8)()
    assert lib.setd_tucker_apply(ctypes.c_void_p(4096), ctypes.c_void_p(8192), 8, huge, M8, 1.0, 0.0, 0, None, 0,
                                 None) == _lib.SETD_EINVAL
    assert b"elements" in lib.setd_last_error()
    out = (ctypes.c_double * 4)()
    assert lib.setd_field_norms(None, None, 10, out, None) == _lib.SETD_EINVAL
    # batch: bad sizes, NULL matrices, reduced precision (FP64 only)
    bd = (ctypes.c_int64 * 4)(16, 16, 1, 16)
    BA = (ctypes.c_void_p * 8)(*([1] * 8))
    assert lib.setd_batch_create(ctypes.byref(h), 0, 2, bd, 2, BA, 0.01, 0, None) == _lib.SETD_EINVAL
    assert lib.setd_batch_create(ctypes.byref(h), 65537, 2, bd, 2, BA, 0.01, 0, None) == _lib.SETD_EINVAL
    assert lib.setd_batch_create(ctypes.byref(h), 2, 2, bd, 2, BA, 0.01, 0, None) == _lib.SETD_EINVAL   # n = 1
    bd[2] = 16
    assert lib.setd_batch_create(ctypes.byref(h), 2, 2, bd, 2, (ctypes.c_void_p * 8)(), 0.01, 0,
                                 None) == _lib.SETD_EINVAL
    assert lib.setd_batch_create(ctypes.byref(h), 2, 2, bd, 2, BA, 0.01, _lib.PREC_F32,
                                 None) == _lib.SETD_EUNSUPPORTED
    assert lib.setd_batch_step(None, None, 1, 0, p, 0, None) == _lib.SETD_EINVAL
    assert lib.setd_etd_step_record(None, None, 0.01, 0, p, 0, None, None) == _lib.SETD_EINVAL
    assert lib.setd_etd_adjoint_step_recorded(None, None, None, None, 0, p, 0, 0, None, None) == _lib.SETD_EINVAL
    info = (ctypes.c_int64 * _lib.BATCH_INFO)()
    assert lib.setd_batch_info(None, info) == _lib.SETD_EINVAL
    assert lib.setd_batch_set_tiles(None, (ctypes.c_int * 6)(2, 2, 0, 2, 2, 0)) == _lib.SETD_EINVAL


def test_python_binding_raises_on_error():
    with pytest.raises(_lib.SetdError) as ei:
        _lib.check(_lib.load().setd_phi_matrices(None, 4, 0.1, 1, None, None))
    assert ei.value.code == _lib.SETD_EINVAL
