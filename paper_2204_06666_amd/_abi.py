"""ctypes declarations of the C ABI in include/ehyb.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libehyb.so")

c_i32, c_i64, c_u32, c_u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
c_vp, c_size = ctypes.c_void_p, ctypes.c_size_t

EHYB_OK, EHYB_EINVAL, EHYB_ENOMEM, EHYB_EUNSUPPORTED, EHYB_EDEVICE, EHYB_ESTATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "EHYB_OK", -1: "EHYB_EINVAL", -2: "EHYB_ENOMEM", -3: "EHYB_EUNSUPPORTED",
                -4: "EHYB_EDEVICE", -5: "EHYB_ESTATE"}
EHYB_F64, EHYB_F32, EHYB_BF16, EHYB_F32_ACC64, EHYB_BF16_ACC64 = 0, 1, 2, 3, 4
EHYB_VEC_PERMUTED = 1
EHYB_LOAD_AUTO, EHYB_LOAD_CACHED, EHYB_LOAD_STREAM = 0, 1, 2


class CsrHost(ctypes.Structure):
    _fields_ = [("n_rows", c_i64), ("n_cols", c_i64), ("nnz", c_i64),
                ("row_ptr", c_vp), ("col_idx", c_vp), ("val", c_vp)]


class Params(ctypes.Structure):
    _fields_ = [("slice_rows", c_i32), ("ell_width_cap", c_i32), ("rows_per_wave", c_i32),
                ("value_dtype", c_i32), ("lds_bytes", c_i32), ("num_cus", c_i32),
                ("n_threads", c_i32), ("imbalance_pct", c_i32), ("partitioner", c_i32),
                ("halo_rows", c_i32), ("n_rhs", c_i32), ("reserved", c_i32), ("seed", c_u64)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n", c_i64), ("nnz", c_i64), ("nnz_ell", c_i64), ("nnz_er", c_i64),
                ("ell_slots", c_i64), ("er_slots", c_i64), ("n_er_rows", c_i64),
                ("nnz_halo", c_i64), ("n_halo", c_i64),
                ("device_bytes", c_i64), ("algorithmic_bytes", c_i64),
                ("nparts", c_i32), ("nslices", c_i32), ("ner_slices", c_i32), ("slice_rows", c_i32),
                ("max_part_rows", c_i32), ("rows_per_slice", c_i32), ("lanes_per_row", c_i32),
                ("kc", c_i32), ("value_dtype", c_i32), ("eq1_K", c_i32),
                ("max_halo", c_i32), ("lds_bytes_used", c_i32), ("n_rhs", c_i32), ("n_er_wide", c_i32),
                ("ell_width_cap", c_i32), ("n_er_pieces", c_i32),
                ("t_graph_s", ctypes.c_double), ("t_partition_s", ctypes.c_double),
                ("t_reorder_s", ctypes.c_double), ("t_encode_s", ctypes.c_double)]


class PlanArrays(ctypes.Structure):
    _fields_ = [("n", c_i64), ("nparts", c_i32), ("nslices", c_i32), ("ner_slices", c_i32),
                ("lanes_per_row", c_i32), ("kc", c_i32), ("value_dtype", c_i32),
                ("ell_slots", c_i64), ("er_slots", c_i64), ("n_halo", c_i64),
                ("perm", c_vp), ("part_start", c_vp), ("slice_start", c_vp), ("er_slice_start", c_vp),
                ("ell_free", c_vp), ("halo_start", c_vp), ("halo_idx", c_vp),
                ("ell_meta", c_vp), ("er_meta", c_vp), ("er_row", c_vp),
                ("ell_val", c_vp), ("ell_col", c_vp), ("er_val", c_vp), ("er_col", c_vp),
                ("row_ell_len", c_vp), ("row_er_len", c_vp)]


class DeviceInfo(ctypes.Structure):
    _fields_ = [("device", c_i32), ("num_cus", c_i32), ("lds_per_block", c_i32),
                ("warp_size", c_i32), ("clock_khz", c_i32), ("mem_clock_khz", c_i32),
                ("mem_bus_width", c_i32), ("l2_bytes", c_i32), ("arch", ctypes.c_char * 64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "ehyb_preprocess": (c_i32, [ctypes.POINTER(CsrHost), ctypes.POINTER(Params), ctypes.POINTER(c_vp)]),
    "ehyb_preprocess_partitioned": (c_i32, [ctypes.POINTER(CsrHost), ctypes.POINTER(Params), c_vp, c_i32,
                                            ctypes.POINTER(c_vp)]),
    "ehyb_features": (c_i32, [ctypes.POINTER(CsrHost), c_i32, c_vp]),
    "ehyb_mlp_forward": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "ehyb_mlp_workspace_bytes": (c_i32, [c_i32, ctypes.POINTER(ctypes.c_size_t)]),
    "ehyb_mlp_grad": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "ehyb_mlp_grad_noalloc": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "ehyb_mlp_adam": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.c_float, c_vp]),
    "ehyb_plan_stats_get": (c_i32, [c_vp, ctypes.POINTER(PlanStats)]),
    "ehyb_plan_arrays_get": (c_i32, [c_vp, ctypes.POINTER(PlanArrays)]),
    "ehyb_plan_decode_csr": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "ehyb_plan_device_bytes": (c_i32, [c_vp, ctypes.POINTER(c_size)]),
    "ehyb_plan_upload": (c_i32, [c_vp, c_vp, c_size, c_vp]),
    "ehyb_spmv": (c_i32, [c_vp, c_vp, c_vp, c_u32, c_vp]),
    "ehyb_plan_set_launch": (c_i32, [c_vp, c_i32]),
    "ehyb_plan_set_load_mode": (c_i32, [c_vp, c_i32]),
    "ehyb_batch_set_load_mode": (c_i32, [c_vp, c_i32]),
    "ehyb_permute_x": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "ehyb_unpermute_y": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "ehyb_plan_save": (c_i32, [c_vp, ctypes.c_char_p]),
    "ehyb_plan_load": (c_i32, [ctypes.c_char_p, ctypes.POINTER(c_vp)]),
    "ehyb_plan_destroy": (None, [c_vp]),
    "ehyb_csr_spmv_f64": (c_i32, [c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp]),
    "ehyb_probe_read": (c_i32, [c_vp, c_size, c_vp, c_vp]),
    "ehyb_cache_flush": (c_i32, [c_vp, c_size, c_vp, c_vp]),
    "ehyb_probe_copy": (c_i32, [c_vp, c_vp, c_size, c_vp]),
    "ehyb_device_info_get": (c_i32, [ctypes.POINTER(DeviceInfo)]),
    "ehyb_batch_create": (c_i32, [ctypes.POINTER(c_vp), c_i32, c_i32, ctypes.POINTER(c_vp)]),
    "ehyb_batch_device_bytes": (c_i32, [c_vp, ctypes.POINTER(c_size)]),
    "ehyb_batch_upload": (c_i32, [c_vp, c_vp, c_size, c_vp]),
    "ehyb_spmm_batched": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp), c_u32, c_vp]),
    "ehyb_batch_destroy": (None, [c_vp]),
    "ehyb_last_error": (ctypes.c_char_p, []),
    "ehyb_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libehyb.so (built in-tree).  There is no fallback: without the
    library nothing in this package can run."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"EHYB native library not found at {LIB_PATH}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)")
    # The library and torch must share one HIP runtime.  torch ships its own
    # libamdhip64 (soname libamdhip64.so.7); once torch is imported, the
    # library's dependency on that soname resolves to torch's copy.  Loading
    # the library first would bring in a second runtime, which does not see
    # torch's devices or allocations.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class EhybError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


def check(status: int, where: str):
    if status != EHYB_OK:
        msg = load().ehyb_last_error()
        raise EhybError(status, where, msg.decode() if msg else "")
