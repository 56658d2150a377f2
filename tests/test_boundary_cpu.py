"""The C ABI library loads and exports what include/pcdm.h declares; argument
checks that return before any device call.  No compute runs here."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1212_0873_amd as pc
from paper_1212_0873_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pcdm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pcdm_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(_lib.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = pc.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_last_error_is_empty_string_initially():
    assert isinstance(pc.load().pcdm_last_error(), bytes)


def _desc(m=4, n=3, nnz=3, dtype=_lib.PCDM_F64):
    cp = np.arange(n + 1, dtype=np.int64)
    ri = np.zeros(max(nnz, 1), dtype=np.int32)
    v = np.ones(max(nnz, 1))
    d = _lib.pcdm_csc(m, n, nnz, cp.ctypes.data, ri.ctypes.data, v.ctypes.data, dtype, 0)
    return d, (cp, ri, v)


@pytest.mark.parametrize("field,value,lam,tau", [
    ("m", 0, 0.1, 1), ("n", 0, 0.1, 1), ("nnz", 1, 0.1, 1), ("dtype", 7, 0.1, 1),
    (None, None, -1.0, 1), (None, None, float("nan"), 1), (None, None, 0.1, 0), (None, None, 0.1, 4),
])
def test_create_rejects_bad_scalars(field, value, lam, tau):
    lib = pc.load()
    d, keep = _desc()
    if field:
        setattr(d, field, value)
    b = np.zeros(4)
    h = ctypes.c_void_p(1234)
    st = lib.pcdm_create(ctypes.byref(d), b.ctypes.data, lam, tau, 0, ctypes.byref(h))
    assert st == _lib.PCDM_EINVAL
    assert h.value is None
    assert lib.pcdm_last_error()


def test_null_arguments_rejected():
    lib = pc.load()
    assert lib.pcdm_create(None, None, 0.1, 1, 0, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_step(None, 1, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_set_option(None, b"tau", 1.0) == _lib.PCDM_EINVAL
    assert lib.pcdm_objective(None, None, None, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_get_x(None, None, 0, 0, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_set_x(None, None, 0, 0, 0, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_get_residual(None, None, 0, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_sample(0, 0, 1, 1, None, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_sample(0, 0, 5, 4, 8, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_destroy(None) == _lib.PCDM_OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()
