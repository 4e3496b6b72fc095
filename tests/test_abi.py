"""The C ABI library: loads, exports what include/bdc.h declares, and checks
its arguments on the host (no device work; runs without a GPU)."""

import ctypes
import os
import re

import pytest

from paper_2508_11467_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bdc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(bdc_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_header_functions_are_exported(lib):
    names = declared_functions()
    assert "bdc_svd" in names and "bdc_svd_batched" in names and "bdc_create" in names
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares each of them
    assert set(names) == set(_lib.SIGNATURES)


def test_default_options(lib):
    o = _lib.Options()
    lib.bdc_default_options(ctypes.byref(o))
    assert o.leaf_size == 32 and o.max_secular_iters == 64 and o.timing == 0


def test_null_handle_rejected(lib):
    assert lib.bdc_svd(None, 4, None, None, None, None, None, None) == _lib.BDC_ERR_INVALID_HANDLE
    assert lib.bdc_destroy(None) == _lib.BDC_ERR_INVALID_HANDLE
    assert lib.bdc_get_info(None, None, None) == _lib.BDC_ERR_INVALID_HANDLE
    assert lib.bdc_step_gemm(None, 1, 1, 1, None, 1, None, 1, None, 1, None) == _lib.BDC_ERR_INVALID_HANDLE


def test_dense_stage_entry_points_reject_a_null_handle(lib):
    """The entry points around the bidiagonal solve check the handle before
    touching any pointer (no GPU needed)."""
    bad = _lib.BDC_ERR_INVALID_HANDLE
    assert lib.bdc_geqrf(None, 4, 4, None, 4, None, 0, None) == bad
    assert lib.bdc_orgqr(None, 4, 4, 4, None, 4, None, None, 4, 0, None) == bad
    assert lib.bdc_gebrd(None, 4, 4, None, 4, None, None, None, None, 0, None) == bad
    assert lib.bdc_apply_reflectors(None, 0, 4, 4, 4, 0, None, 1, 4, None, None, 4, 0, None) == bad
    assert lib.bdc_apply_reflectors_noalloc(None, 0, 4, 4, 4, 0, None, 1, 4, None, None, 4, 0, None) == bad
    assert lib.bdc_step_gemm(None, 4, 4, 4, None, 4, None, 4, None, 4, None) == bad


def test_create_validates_options(lib):
    h = ctypes.c_void_p()
    assert lib.bdc_create(None, 0, None) == -1
    for field, bad in (("leaf_size", 3), ("leaf_size", 33), ("max_secular_iters", 1), ("max_leaf_sweeps", 0)):
        o = _lib.Options()
        lib.bdc_default_options(ctypes.byref(o))
        setattr(o, field, bad)
        assert lib.bdc_create(ctypes.byref(h), 0, ctypes.byref(o)) == -3


def test_create_without_device(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except Exception:
        pass
    h = ctypes.c_void_p()
    assert lib.bdc_create(ctypes.byref(h), 0, None) == _lib.BDC_ERR_NO_DEVICE
    assert lib.bdc_create(ctypes.byref(h), -1, None) == _lib.BDC_ERR_NO_DEVICE


def test_status_strings(lib):
    for code in (0, -1001, -1002, -1003, -1004, -1005, -1006, -3, 5):
        assert len(_lib.status_string(code)) > 0
