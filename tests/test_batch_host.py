"""Batch construction through the C ABI (host only, no GPU)."""
import ctypes

import pytest

import matgen
from paper_2204_06666_amd import EhybError, Plan, _abi


def _create(plans, n_rhs):
    lib = _abi.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    st = lib.ehyb_batch_create(arr, len(plans), n_rhs, ctypes.byref(h))
    if st == 0:
        lib.ehyb_batch_destroy(h)
    return st


def test_batch_validation():
    A = matgen.poisson2d(16)
    B = matgen.stencil3d(6)
    p8 = [Plan(A, n_rhs=8, value_dtype=1), Plan(B, n_rhs=8, value_dtype=1)]
    assert _create(p8, 8) == _abi.EHYB_OK
    assert _create(p8, 4) == _abi.EHYB_EINVAL                      # built for another n_rhs
    assert _create(p8, 3) == _abi.EHYB_EINVAL
    mixed = [Plan(A, n_rhs=8, value_dtype=1), Plan(B, n_rhs=8, value_dtype=0)]
    assert _create(mixed, 8) == _abi.EHYB_EINVAL                   # value types differ
    rpw = [Plan(A, n_rhs=2, rows_per_wave=32), Plan(B, n_rhs=2, rows_per_wave=32)]
    assert _create(rpw, 2) == _abi.EHYB_EUNSUPPORTED               # no batched kernel for L = 2
    lib = _abi.load()
    h = ctypes.c_void_p()
    assert lib.ehyb_batch_create(None, 0, 8, ctypes.byref(h)) == _abi.EHYB_EINVAL
    many = (ctypes.c_void_p * 129)(*([p8[0].handle.value] * 129))
    assert lib.ehyb_batch_create(many, 129, 8, ctypes.byref(h)) == _abi.EHYB_EINVAL


def test_batch_upload_needs_uploaded_plans():
    A = matgen.poisson2d(16)
    P = Plan(A, n_rhs=4)
    lib = _abi.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 1)(P.handle.value)
    assert lib.ehyb_batch_create(arr, 1, 4, ctypes.byref(h)) == _abi.EHYB_OK
    try:
        assert lib.ehyb_batch_upload(h, ctypes.c_void_p(4096), 1 << 20, None) == _abi.EHYB_ESTATE
        xs = (ctypes.c_void_p * 1)(4096)
        assert lib.ehyb_spmm_batched(h, 4, xs, xs, 1, None) == _abi.EHYB_ESTATE
    finally:
        lib.ehyb_batch_destroy(h)


def test_n_rhs_shrinks_partitions():
    """The LDS budget holds n_rhs elements per row (tau of Eq. 1 grows
    n_rhs-fold), so a plan for more right-hand sides gets shorter partitions."""
    A = matgen.stencil3d(40)
    lds = 32 * 1024
    s1 = Plan(A, n_rhs=1, lds_bytes=lds).stats()
    s8 = Plan(A, n_rhs=8, lds_bytes=lds).stats()
    assert s8["n_rhs"] == 8 and s1["n_rhs"] == 1
    assert s1["slice_rows"] == 512 and s8["slice_rows"] == (lds - 64) // (2 * 8 * 8)
    assert s8["max_part_rows"] * 2 * 8 * 8 <= lds - 64
    with pytest.raises(EhybError):
        Plan(A, n_rhs=3)
