"""EHYB (explicit-caching hybrid) SpMV for AMD MI355X (gfx950).

Thin Python binding of the C ABI in ``include/ehyb.h``: every step of
preprocessing and of the product runs in the native library (host C++ and HIP
kernels); this module only marshals arguments.  PyTorch supplies device memory
and streams.

    plan = Plan(A, slice_rows=0, rows_per_wave=64)   # host preprocessing
    plan.upload("cuda:0")                             # device blob (torch-owned)
    y = plan.spmv(x)                                  # y = A x on the GPU
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _abi
from ._abi import (EHYB_BF16, EHYB_BF16_ACC64, EHYB_F32, EHYB_F32_ACC64, EHYB_F64,  # noqa: F401
                   EHYB_LOAD_AUTO, EHYB_LOAD_CACHED,
                   EHYB_LOAD_STREAM, EHYB_VEC_PERMUTED, EhybError,
                   check, load)

__all__ = ["Plan", "Batch", "csr_spmv", "probe_read", "cache_flush", "probe_copy", "device_info", "version",
           "EhybError", "EHYB_F64", "EHYB_F32", "EHYB_BF16", "EHYB_F32_ACC64", "EHYB_BF16_ACC64",
           "EHYB_VEC_PERMUTED", "EHYB_LOAD_AUTO",
           "EHYB_LOAD_CACHED", "EHYB_LOAD_STREAM", "load"]

_NP_VAL = {EHYB_F64: np.float64, EHYB_F32: np.float32, EHYB_BF16: np.uint16,
           EHYB_F32_ACC64: np.float32, EHYB_BF16_ACC64: np.uint16}


def version() -> str:
    return load().ehyb_version().decode()


def _ptr(a) -> ctypes.c_void_p:
    """Address of a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _as_csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, ci, v


class Plan:
    """An EHYB plan: the host preprocessing (Alg. 1-2) of one square matrix.

    Keyword parameters mirror ``ehyb_params`` (zero = default)."""

    def __init__(self, A=None, *, slice_rows: int = 0, ell_width_cap: int = 0,
                 rows_per_wave: int = 0, value_dtype: int = EHYB_F64, lds_bytes: int = 0,
                 num_cus: int = 0, n_threads: int = 0, imbalance_pct: int = 0,
                 partitioner: int = 0, halo_rows: int = 0, n_rhs: int = 0, seed: int = 0,
                 partition=None, _handle=None):
        self._lib = load()
        self._h = ctypes.c_void_p()
        self._blob = None
        if _handle is not None:
            self._h = _handle
            st = self.stats()
            self.n, self.value_dtype = st["n"], st["value_dtype"]
            return
        rp, ci, v = _as_csr(A)
        csr = _abi.CsrHost(A.n_rows, A.n_cols, int(rp[-1]) if rp.size else 0,
                           rp.ctypes.data, ci.ctypes.data if ci.size else None,
                           v.ctypes.data if v.size else None)
        prm = _abi.Params(slice_rows, ell_width_cap, rows_per_wave, value_dtype, lds_bytes,
                          num_cus, n_threads, imbalance_pct, partitioner, halo_rows, n_rhs, 0, seed)
        if partition is None:
            check(self._lib.ehyb_preprocess(ctypes.byref(csr), ctypes.byref(prm), ctypes.byref(self._h)),
                  "ehyb_preprocess")
        else:
            part = np.ascontiguousarray(partition, dtype=np.int32)
            if part.shape != (A.n_rows,):
                raise ValueError("partition must hold one id per row")
            k = int(part.max()) + 1 if part.size else 0
            check(self._lib.ehyb_preprocess_partitioned(ctypes.byref(csr), ctypes.byref(prm),
                                                        part.ctypes.data if part.size else None, k,
                                                        ctypes.byref(self._h)), "ehyb_preprocess_partitioned")
        self.n = int(A.n_rows)
        self.value_dtype = int(value_dtype)

    # ------------------------------------------------------------ host side
    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.ehyb_plan_destroy(h)
            self._h = ctypes.c_void_p()

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def stats(self) -> dict:
        st = _abi.PlanStats()
        check(self._lib.ehyb_plan_stats_get(self._h, ctypes.byref(st)), "ehyb_plan_stats_get")
        return {f: getattr(st, f) for f, _ in st._fields_ if not f.startswith("reserved")}

    def arrays(self) -> dict:
        """Copies of the plan's host arrays (the layout of include/ehyb.h)."""
        ar = _abi.PlanArrays()
        check(self._lib.ehyb_plan_arrays_get(self._h, ctypes.byref(ar)), "ehyb_plan_arrays_get")
        n, nparts, ns = ar.n, ar.nparts, ar.nslices
        vt = _NP_VAL[ar.value_dtype]

        def grab(addr, count, dtype):
            if count == 0:
                return np.zeros(0, dtype=dtype)
            buf = (ctypes.c_char * (count * np.dtype(dtype).itemsize)).from_address(addr)
            return np.frombuffer(buf, dtype=dtype).copy()

        C = 64 // ar.lanes_per_row
        nes = ar.ner_slices
        return dict(
            n=n, nparts=nparts, L=ar.lanes_per_row, kc=ar.kc, value_dtype=ar.value_dtype,
            perm=grab(ar.perm, n, np.int32), part_start=grab(ar.part_start, nparts + 1, np.int32),
            slice_start=grab(ar.slice_start, nparts + 1, np.int32),
            er_slice_start=grab(ar.er_slice_start, nparts + 1, np.int32),
            ell_free=grab(ar.ell_free, nparts, np.int32),
            halo_start=grab(ar.halo_start, nparts + 1, np.int32),
            halo_idx=grab(ar.halo_idx, ar.n_halo, np.int32),
            ell_meta=grab(ar.ell_meta, 4 * ns, np.uint32).reshape(ns, 4),
            er_meta=grab(ar.er_meta, 2 * nes, np.uint32).reshape(nes, 2),
            er_row=grab(ar.er_row, C * nes, np.uint16).reshape(nes, C),
            ell_val=grab(ar.ell_val, ar.ell_slots, vt), ell_col=grab(ar.ell_col, ar.ell_slots, np.uint16),
            er_val=grab(ar.er_val, ar.er_slots, vt), er_col=grab(ar.er_col, ar.er_slots, np.int32),
            row_ell_len=grab(ar.row_ell_len, n, np.int32), row_er_len=grab(ar.row_er_len, n, np.int32))

    def perm(self) -> np.ndarray:
        return self.arrays()["perm"]

    def partition(self) -> np.ndarray:
        """Partition id of every original row (from perm and part_start)."""
        a = self.arrays()
        part = np.empty(self.n, dtype=np.int32)
        ps = a["part_start"]
        part[a["perm"]] = np.repeat(np.arange(ps.size - 1, dtype=np.int32), np.diff(ps))
        return part

    def decode(self):
        """CSR of P A P^T (row_ptr int64, col int32, val float64)."""
        st = self.stats()
        n, nnz = st["n"], st["nnz"]
        rp = np.zeros(n + 1, dtype=np.int64)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1), dtype=np.float64)
        check(self._lib.ehyb_plan_decode_csr(self._h, _ptr(rp), _ptr(ci), _ptr(v)), "decode")
        return rp, ci[:nnz], v[:nnz]

    def save(self, path: str):
        check(self._lib.ehyb_plan_save(self._h, path.encode()), "ehyb_plan_save")

    @classmethod
    def load(cls, path: str) -> "Plan":
        lib = load()
        h = ctypes.c_void_p()
        check(lib.ehyb_plan_load(path.encode(), ctypes.byref(h)), "ehyb_plan_load")
        return cls(_handle=h)

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        check(self._lib.ehyb_plan_device_bytes(self._h, ctypes.byref(b)), "device_bytes")
        return b.value

    def set_launch(self, waves_per_wg: int = 0):
        """Wavefronts per workgroup of spmv (0 = library choice); results are unchanged."""
        check(self._lib.ehyb_plan_set_launch(self._h, waves_per_wg), "set_launch")
        return self

    def set_load_mode(self, mode: int = 0):
        """EHYB_LOAD_AUTO / _CACHED / _STREAM loads of the value and column arrays."""
        check(self._lib.ehyb_plan_set_load_mode(self._h, mode), "set_load_mode")
        return self

    # ---------------------------------------------------------- device side
    def upload(self, device="cuda:0", stream=None):
        """Allocate the device blob with torch and copy the plan into it."""
        import torch
        nbytes = self.device_bytes()
        blob = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-blob.data_ptr()) % 256
        view = blob[off:off + nbytes]
        with torch.cuda.device(blob.device):
            check(self._lib.ehyb_plan_upload(self._h, ctypes.c_void_p(view.data_ptr()), nbytes,
                                             _stream(stream)), "ehyb_plan_upload")
        self._blob = blob
        self.device = blob.device
        return self

    @property
    def x_dtype(self):
        """torch dtype of x and y: float64 for FP64 plans, float32 otherwise."""
        import torch
        return torch.float64 if self.value_dtype == EHYB_F64 else torch.float32

    def spmv(self, x, y=None, permuted: bool = True, stream=None):
        """y = A x.  ``permuted``: x and y are in the plan's order."""
        import torch
        n = self.n
        if y is None:
            y = torch.empty(n, dtype=x.dtype, device=x.device)
        want = self.x_dtype
        for t in (x, y):
            if t.dtype != want or not t.is_contiguous() or t.numel() != n or not t.is_cuda:
                raise ValueError(f"x and y must be contiguous {want} CUDA tensors of length n")
        check(self._lib.ehyb_spmv(self._h, _ptr(x), _ptr(y), EHYB_VEC_PERMUTED if permuted else 0,
                                  _stream(stream)), "ehyb_spmv")
        return y

    def permute_x(self, x, xp=None, stream=None):
        import torch
        xp = torch.empty_like(x) if xp is None else xp
        check(self._lib.ehyb_permute_x(self._h, _ptr(x), _ptr(xp), _stream(stream)), "permute_x")
        return xp

    def unpermute_y(self, yp, y=None, stream=None):
        import torch
        y = torch.empty_like(yp) if y is None else y
        check(self._lib.ehyb_unpermute_y(self._h, _ptr(yp), _ptr(y), _stream(stream)), "unpermute_y")
        return y


class Batch:
    """Several uploaded plans (one value type, one rows_per_wave, built for
    `n_rhs`) multiplied in one persistent kernel launch: Y_i = A_i X_i with X_i,
    Y_i row-major [n_i][n_rhs] in each plan's permuted order."""

    def __init__(self, plans, n_rhs: int, device="cuda:0", stream=None):
        import torch
        self._lib = load()
        self.plans = list(plans)          # keep the plans (and their blobs) alive
        self.n_rhs = int(n_rhs)
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        check(self._lib.ehyb_batch_create(arr, len(self.plans), self.n_rhs, ctypes.byref(self._h)),
              "ehyb_batch_create")
        b = ctypes.c_size_t()
        check(self._lib.ehyb_batch_device_bytes(self._h, ctypes.byref(b)), "ehyb_batch_device_bytes")
        blob = torch.empty(b.value + 256, dtype=torch.uint8, device=device)
        off = (-blob.data_ptr()) % 256
        with torch.cuda.device(blob.device):
            check(self._lib.ehyb_batch_upload(self._h, ctypes.c_void_p(blob.data_ptr() + off), b.value,
                                              _stream(stream)), "ehyb_batch_upload")
        self._blob = blob

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.ehyb_batch_destroy(h)
            self._h = ctypes.c_void_p()

    def set_load_mode(self, mode: int = 0):
        """EHYB_LOAD_AUTO / _CACHED / _STREAM loads of the value and column arrays."""
        check(self._lib.ehyb_batch_set_load_mode(self._h, mode), "set_load_mode")
        return self

    def spmm(self, X, Y, stream=None):
        """Y[i] = A_i X[i] for every matrix (lists of CUDA tensors [n_i, n_rhs])."""
        k = len(self.plans)
        if len(X) != k or len(Y) != k:
            raise ValueError("one X and one Y per matrix")
        for p, x, y in zip(self.plans, X, Y):
            for t in (x, y):
                if (t.dtype != p.x_dtype or not t.is_contiguous() or not t.is_cuda
                        or tuple(t.shape) != (p.n, self.n_rhs)):
                    raise ValueError("X[i], Y[i] must be contiguous [n_i, n_rhs] CUDA tensors of the plan's dtype")
        xs = (ctypes.c_void_p * k)(*[x.data_ptr() for x in X])
        ys = (ctypes.c_void_p * k)(*[y.data_ptr() for y in Y])
        check(self._lib.ehyb_spmm_batched(self._h, self.n_rhs, xs, ys, EHYB_VEC_PERMUTED, _stream(stream)),
              "ehyb_spmm_batched")
        return Y


def features(A, n_threads: int = 0) -> np.ndarray:
    """The 32 sparsity features of A (float32), as defined by ehyb_features."""
    rp, ci, v = _as_csr(A)
    csr = _abi.CsrHost(A.n_rows, A.n_cols, int(rp[-1]) if rp.size else 0, rp.ctypes.data,
                       ci.ctypes.data if ci.size else None, v.ctypes.data if v.size else None)
    out = np.zeros(32, dtype=np.float32)
    check(load().ehyb_features(ctypes.byref(csr), n_threads, out.ctypes.data), "ehyb_features")
    return out


def csr_spmv(row_ptr32, col, val, x, y, lanes_per_row: int = 0, stream=None):
    """Plain CSR y = A x on the device (int32 row pointers)."""
    n = row_ptr32.numel() - 1
    check(load().ehyb_csr_spmv_f64(n, col.numel(), _ptr(row_ptr32), _ptr(col), _ptr(val), _ptr(x),
                                   _ptr(y), lanes_per_row, _stream(stream)), "ehyb_csr_spmv_f64")
    return y


def probe_read(buf, sink, stream=None):
    check(load().ehyb_probe_read(_ptr(buf), buf.numel() * buf.element_size(), _ptr(sink),
                                 _stream(stream)), "probe_read")


def cache_flush(buf, sink, stream=None):
    """Read ``buf`` with cache-allocating loads (evicts L2 and the Infinity Cache)."""
    check(load().ehyb_cache_flush(_ptr(buf), buf.numel() * buf.element_size(), _ptr(sink),
                                  _stream(stream)), "cache_flush")


def probe_copy(src, dst, stream=None):
    check(load().ehyb_probe_copy(_ptr(src), _ptr(dst), src.numel() * src.element_size(),
                                 _stream(stream)), "probe_copy")


def device_info() -> dict:
    di = _abi.DeviceInfo()
    check(load().ehyb_device_info_get(ctypes.byref(di)), "device_info")
    d = {f: getattr(di, f) for f, _ in di._fields_}
    d["arch"] = di.arch.decode()
    return d
