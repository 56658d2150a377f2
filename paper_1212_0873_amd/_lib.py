"""ctypes declarations of the C ABI in include/pcdm.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcdm.so")

PCDM_OK, PCDM_EINVAL, PCDM_ENOMEM, PCDM_EDEVICE, PCDM_ESTATE, PCDM_ENOTCONV = 0, -1, -2, -3, -4, -5
PCDM_F32, PCDM_BF16, PCDM_F64 = 0, 1, 2
STATUS_NAMES = {0: "PCDM_OK", -1: "PCDM_EINVAL", -2: "PCDM_ENOMEM", -3: "PCDM_EDEVICE",
                -4: "PCDM_ESTATE", -5: "PCDM_ENOTCONV"}

# every symbol include/pcdm.h declares
EXPORTS = ("pcdm_create", "pcdm_destroy", "pcdm_last_error", "pcdm_set_option", "pcdm_get_info",
           "pcdm_step", "pcdm_objective", "pcdm_get_x", "pcdm_set_x", "pcdm_get_residual",
           "pcdm_grad_backward", "pcdm_grad_backward_noalloc", "pcdm_set_rhs", "pcdm_kernel_time",
           "pcdm_autotune", "pcdm_sample",
           "pcdm_sample_draw", "pcdm_set_slot_mask", "pcdm_step_async", "pcdm_create_model",
           "pcdm_create_group",
           "pcdm_batch_create", "pcdm_batch_step", "pcdm_batch_objective", "pcdm_batch_set_active",
           "pcdm_batch_get_x", "pcdm_batch_get_info", "pcdm_batch_set_option", "pcdm_batch_autotune",
           "pcdm_batch_destroy")


class pcdm_csc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("dtype", ctypes.c_int32), ("on_device", ctypes.c_int32)]


class pcdm_info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("tau", ctypes.c_int64), ("k", ctypes.c_int64), ("omega", ctypes.c_int64),
                ("refresh_every", ctypes.c_int64), ("nonzero_updates", ctypes.c_int64),
                ("stored_nnz", ctypes.c_int64), ("beta", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("atb_inf", ctypes.c_double), ("dtype", ctypes.c_int32), ("beta_rule", ctypes.c_int32),
                ("lanes_per_column", ctypes.c_int32), ("chunks_per_lane", ctypes.c_int32),
                ("sampling", ctypes.c_int32), ("gather_route", ctypes.c_int32), ("binomial_p", ctypes.c_double),
                ("expected_set_size", ctypes.c_double), ("mask_len", ctypes.c_int64),
                ("narrow_below", ctypes.c_int64), ("nblocks", ctypes.c_int64), ("loss", ctypes.c_int32),
                ("scatter_route", ctypes.c_int32),
                ("loss_scale", ctypes.c_double), ("l2", ctypes.c_double), ("linear", ctypes.c_double),
                ("lower", ctypes.c_double), ("upper", ctypes.c_double), ("async_picks", ctypes.c_int64),
                ("async_processors", ctypes.c_int64),
                ("max_incremental", ctypes.c_int64),
                ("max_candidates", ctypes.c_int64)]


class pcdm_model(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_int32), ("reserved", ctypes.c_int32), ("scale", ctypes.c_double),
                ("l1", ctypes.c_double), ("l2", ctypes.c_double), ("linear", ctypes.c_double),
                ("lower", ctypes.c_double), ("upper", ctypes.c_double)]


class PCDMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lock = threading.Lock()
_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                              "(run __graft_entry__.build() or python paper_1212_0873_amd/build.py)")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        sig = {
            "pcdm_create": [ctypes.POINTER(pcdm_csc), vp, f64, i64, u64, ctypes.POINTER(vp)],
            "pcdm_destroy": [vp],
            "pcdm_create_model": [ctypes.POINTER(pcdm_csc), vp, ctypes.POINTER(pcdm_model), i64, u64,
                                  ctypes.POINTER(vp)],
            "pcdm_create_group": [ctypes.POINTER(pcdm_csc), vp, f64, vp, i64, i64, u64, ctypes.POINTER(vp)],
            "pcdm_set_option": [vp, ctypes.c_char_p, f64],
            "pcdm_get_info": [vp, ctypes.POINTER(pcdm_info)],
            "pcdm_step": [vp, i64, vp],
            "pcdm_step_async": [vp, i64, vp],
            "pcdm_objective": [vp, pd, pd, vp],
            "pcdm_get_x": [vp, vp, i32, i32, vp],
            "pcdm_set_x": [vp, vp, i32, i32, i64, vp],
            "pcdm_get_residual": [vp, vp, i32, vp],
            "pcdm_grad_backward": [vp, vp, vp, pd, i32, vp],
            "pcdm_grad_backward_noalloc": [vp, vp, vp, pd, vp],
            "pcdm_sample": [u64, u64, i64, i64, vp, vp],
            "pcdm_sample_draw": [i32, f64, u64, u64, i64, i64, vp, vp],
            "pcdm_set_slot_mask": [vp, vp, i64, i32, vp],
            "pcdm_kernel_time": [vp, ctypes.c_char_p, ctypes.POINTER(i64), pd],
            "pcdm_set_rhs": [vp, vp, i32, vp],
            "pcdm_autotune": [vp, i64, vp],
            "pcdm_batch_create": [ctypes.c_int, ctypes.POINTER(pcdm_csc), ctypes.POINTER(vp), pd,
                                  ctypes.POINTER(i64), u64, ctypes.POINTER(vp)],
            "pcdm_batch_step": [vp, i64, vp],
            "pcdm_batch_objective": [vp, pd, pd, vp],
            "pcdm_batch_set_active": [vp, ctypes.POINTER(i32)],
            "pcdm_batch_get_x": [vp, ctypes.c_int, vp, i32, vp],
            "pcdm_batch_get_info": [vp, ctypes.c_int, ctypes.POINTER(pcdm_info)],
            "pcdm_batch_set_option": [vp, ctypes.c_char_p, f64],
            "pcdm_batch_autotune": [vp, i64, vp],
            "pcdm_batch_destroy": [vp],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.pcdm_last_error.argtypes = []
        lib.pcdm_last_error.restype = ctypes.c_char_p
        _lib = lib
        return lib


def check(status: int) -> None:
    if status != PCDM_OK:
        msg = load().pcdm_last_error().decode(errors="replace")
        raise PCDMError(status, msg)
