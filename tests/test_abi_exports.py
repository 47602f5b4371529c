"""The C-ABI library loads and exports every entry point include/ehyb.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2204_06666_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"EHYB_API\s+[\w\s\*]*?\b(ehyb_\w+)\s*\(", text))
    return names


def test_header_declares_the_core_calls():
    names = _declared()
    for core in ("ehyb_preprocess", "ehyb_spmv", "ehyb_plan_upload", "ehyb_plan_decode_csr",
                 "ehyb_csr_spmv_f64", "ehyb_last_error"):
        assert core in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_abi.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert _declared() <= set(_abi.SIGNATURES)


def test_version_and_error_string():
    lib = _abi.load()
    assert lib.ehyb_version().decode().count(".") == 2
    assert isinstance(lib.ehyb_last_error(), bytes)


def test_null_arguments_rejected_without_gpu():
    lib = _abi.load()
    assert lib.ehyb_preprocess(None, None, None) == _abi.EHYB_EINVAL
    assert lib.ehyb_plan_stats_get(None, None) == _abi.EHYB_EINVAL
    assert lib.ehyb_plan_upload(None, None, 0, None) == _abi.EHYB_EINVAL
    assert lib.ehyb_csr_spmv_f64(-1, 0, None, None, None, None, None, 0, None) == _abi.EHYB_EINVAL
    assert lib.ehyb_probe_read(None, 16, None, None) == _abi.EHYB_EINVAL
    assert lib.ehyb_cache_flush(None, 16, None, None) == _abi.EHYB_EINVAL
