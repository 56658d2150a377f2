"""Large synthetic LASSO inputs from the counter-based recipe of
``csrc/gen_common.h``: written on the device for instances too large for the
host, and regenerated entry by entry on the host for checks.

Input construction only (none of the coordinate-descent arithmetic).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import types

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
DEV_LIB = os.path.join(HERE, "libgen_device.so")
HOST_LIB = os.path.join(HERE, "libgen_host.so")
DTYPE_CODE = {"f32": 0, "bf16": 1, "f64": 2}

_dev = None
_host = None


def build() -> None:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = DEV_LIB + f".tmp{os.getpid()}"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", CSRC,
                           os.path.join(CSRC, "gen_device.hip"), "-o", tmp])
    os.replace(tmp, DEV_LIB)
    tmp = HOST_LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-I", CSRC,
                           os.path.join(CSRC, "gen_host.c"), "-o", tmp, "-lm"])
    os.replace(tmp, HOST_LIB)


def _host_lib():
    global _host
    if _host is None:
        if not os.path.exists(HOST_LIB):
            build()
        lib = ctypes.CDLL(HOST_LIB)
        u64, i32, f64, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        lib.gen_host_column_stored.argtypes = [u64, u64, u64, i32, u64, i32, vp, vp]
        lib.gen_host_column_stored.restype = i32
        lib.gen_host_plant.argtypes = [u64, u64, u64, i32, u64, i32, vp, vp, vp]
        lib.gen_host_plant.restype = i32
        lib.gen_host_noise_rows.argtypes = [u64, vp, ctypes.c_int64, f64, vp]
        lib.gen_host_noise_rows.restype = None
        lib.gen_host_csc.argtypes = [u64, u64, u64, i32, i32, vp, vp]
        lib.gen_host_csc.restype = i32
        i64 = ctypes.c_int64
        lib.gen_host_columns.argtypes = [u64, u64, u64, i32, i32, u64, i64, vp, vp, vp, i32]
        lib.gen_host_columns.restype = i32
        lib.gen_host_column_list.argtypes = [u64, u64, u64, i32, i32, vp, i64, vp, vp, vp, i32]
        lib.gen_host_column_list.restype = i32
        lib.gen_host_b.argtypes = [u64, u64, u64, i32, u64, f64, i32, vp, i32]
        lib.gen_host_b.restype = i32
        _host = lib
    return _host


def _dev_lib():
    global _dev
    if _dev is None:
        if not os.path.exists(DEV_LIB):
            raise ImportError(f"device generator not built: {DEV_LIB}")
        lib = ctypes.CDLL(DEV_LIB)
        u64, i32, f64, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        lib.gen_device_instance.argtypes = [u64, u64, u64, i32, u64, f64, i32, vp, vp, vp, vp, vp, vp]
        lib.gen_device_instance.restype = i32
        _dev = lib
    return _dev


def device_instance(m: int, n: int, d: int, K: int, sigma: float, seed: int = 0, dtype: str = "f32"):
    """(A, b, xstar) on the GPU: A has torch tensors col_ptr, row_idx, values."""
    import torch
    vdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f64": torch.float64}[dtype]
    cp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    rows = torch.empty(n * d, dtype=torch.int32, device="cuda")
    vals = torch.empty(n * d, dtype=vdt, device="cuda")
    b = torch.empty(m, dtype=torch.float64, device="cuda")
    xstar = torch.empty(n, dtype=torch.float64, device="cuda")
    st = _dev_lib().gen_device_instance(seed, m, n, d, K, float(sigma), DTYPE_CODE[dtype], cp.data_ptr(),
                                        rows.data_ptr(), vals.data_ptr(), b.data_ptr(), xstar.data_ptr(),
                                        torch.cuda.current_stream().cuda_stream)
    if st != 0:
        raise RuntimeError(f"gen_device_instance failed ({st})")
    A = types.SimpleNamespace(m=m, n=n, col_ptr=cp, row_idx=rows, values=vals)
    return A, b, xstar


def host_column(seed: int, m: int, n: int, d: int, i: int, dtype: str = "f32"):
    """Rows (int32, sorted) and stored values (float64 of the rounded values) of column i."""
    rows = np.empty(d, dtype=np.int32)
    vals = np.empty(d, dtype=np.float64)
    if _host_lib().gen_host_column_stored(seed, m, n, d, i, DTYPE_CODE[dtype], rows.ctypes.data,
                                          vals.ctypes.data) != 0:
        raise ValueError("bad column request")
    return rows, vals


def host_b_at(seed: int, m: int, n: int, d: int, K: int, sigma: float, rows, dtype: str = "f32"):
    """b at the given rows (float64): (A x*)[rows] + noise[rows]."""
    ax = np.zeros(m, dtype=np.float64)
    if _host_lib().gen_host_plant(seed, m, n, d, K, DTYPE_CODE[dtype], ax.ctypes.data, None, None) != 0:
        raise ValueError("bad plant request")
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    noise = np.empty(rows.size, dtype=np.float64)
    _host_lib().gen_host_noise_rows(seed, rows.ctypes.data, rows.size, float(sigma), noise.ctypes.data)
    return ax[rows] + noise


def host_threads() -> int:
    """Worker threads for the host regeneration: the CPUs this process may
    use, at most 16."""
    try:
        cpus = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        cpus = os.cpu_count() or 1
    return max(1, min(16, cpus))


def host_columns(seed: int, m: int, n: int, d: int, i0: int, count: int, dtype: str = "f32",
                 threads: int | None = None):
    """Columns [i0, i0 + count) of the recipe: (col_ptr relative to i0, rows
    int32, stored values as float32).  For f32 / bf16 storage."""
    if dtype == "f64":
        raise ValueError("float32 output holds f32 and bf16 stored values only")
    rows = np.empty(count * d, dtype=np.int32)
    vals = np.empty(count * d, dtype=np.float32)
    if _host_lib().gen_host_columns(seed, m, n, d, DTYPE_CODE[dtype], i0, count, rows.ctypes.data,
                                    vals.ctypes.data, None, threads or host_threads()) != 0:
        raise ValueError("bad column range")
    return np.arange(count + 1, dtype=np.int64) * d, rows, vals


def host_column_list(seed: int, m: int, n: int, d: int, cols, dtype: str = "f32", threads: int | None = None):
    """The given columns (in the given order): (col_ptr, rows int32, stored
    values as float64)."""
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    rows = np.empty(cols.size * d, dtype=np.int32)
    vals = np.empty(cols.size * d, dtype=np.float64)
    if _host_lib().gen_host_column_list(seed, m, n, d, DTYPE_CODE[dtype], cols.ctypes.data, cols.size,
                                        rows.ctypes.data, None, vals.ctypes.data, threads or host_threads()) != 0:
        raise ValueError("bad column list")
    return np.arange(cols.size + 1, dtype=np.int64) * d, rows, vals


def host_b(seed: int, m: int, n: int, d: int, K: int, sigma: float, dtype: str = "f32",
           threads: int | None = None):
    """All of b (float64 [m]) = A x* (stored values) + noise."""
    b = np.empty(m, dtype=np.float64)
    if _host_lib().gen_host_b(seed, m, n, d, K, float(sigma), DTYPE_CODE[dtype], b.ctypes.data,
                              threads or host_threads()) != 0:
        raise ValueError("bad instance request")
    return b


def host_instance(m: int, n: int, d: int, K: int, sigma: float, seed: int = 0, dtype: str = "f32"):
    """The same recipe built entirely on the host (for sizes the host can
    hold): a ``workloads.CSC`` with values stored as ``dtype``, b and x*."""
    from .lasso import CSC
    rows = np.empty(n * d, dtype=np.int32)
    vals = np.empty(n * d, dtype=np.float64)
    if _host_lib().gen_host_csc(seed, m, n, d, DTYPE_CODE[dtype], rows.ctypes.data, vals.ctypes.data) != 0:
        raise ValueError("bad instance request")
    ax = np.zeros(m, dtype=np.float64)
    pos = np.empty(K, dtype=np.uint64)
    xv = np.empty(K, dtype=np.float64)
    _host_lib().gen_host_plant(seed, m, n, d, K, DTYPE_CODE[dtype], ax.ctypes.data, pos.ctypes.data, xv.ctypes.data)
    noise = np.empty(m, dtype=np.float64)
    allrows = np.arange(m, dtype=np.int64)
    _host_lib().gen_host_noise_rows(seed, allrows.ctypes.data, m, float(sigma), noise.ctypes.data)
    xstar = np.zeros(n)
    xstar[pos.astype(np.int64)] = xv
    A = CSC(m, n, np.arange(n + 1, dtype=np.int64) * d, rows, vals)
    if dtype != "f64":
        A = A.astype(dtype)  # values already rounded: exact conversion
    return A, ax + noise, xstar
