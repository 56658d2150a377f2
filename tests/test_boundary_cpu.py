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


def test_new_entry_points_reject_null_and_bad_arguments():
    """Argument checks that run on the host, before any device work."""
    lib = pc.load()
    assert lib.pcdm_step_async(None, 1, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_set_slot_mask(None, None, 0, 0, None) == _lib.PCDM_EINVAL
    assert lib.pcdm_sample_draw(3, 1.0, 0, 0, 4, 10, 8, None) == _lib.PCDM_EINVAL       # unknown sampling
    assert lib.pcdm_sample_draw(2, 0.0, 0, 0, 4, 10, 8, None) == _lib.PCDM_EINVAL       # p_b out of (0, 1]
    assert lib.pcdm_sample_draw(1, 1.0, 0, 0, 4, 10, None, None) == _lib.PCDM_EINVAL    # no output
    d, keep = _desc()
    b = np.zeros(4)
    h = ctypes.c_void_p(1234)
    assert lib.pcdm_create_model(ctypes.byref(d), b.ctypes.data, None, 1, 0, ctypes.byref(h)) == _lib.PCDM_EINVAL
    assert h.value is None


@pytest.mark.parametrize("loss,scale,l1,l2,lin,lo,hi", [
    (3, 1.0, 0.0, 0.0, 0.0, -np.inf, np.inf),          # unknown loss
    (0, 0.0, 0.0, 0.0, 0.0, -np.inf, np.inf),          # scale must be > 0
    (0, np.inf, 0.0, 0.0, 0.0, -np.inf, np.inf),
    (0, 1.0, -0.1, 0.0, 0.0, -np.inf, np.inf),         # negative l1
    (1, 1.0, 0.0, -1.0, 0.0, -np.inf, np.inf),         # negative l2
    (2, 1.0, 0.0, 0.0, np.nan, -np.inf, np.inf),       # linear term not finite
    (0, 1.0, 0.0, 0.0, 0.0, 0.5, 1.0),                 # box must contain 0
    (0, 1.0, 0.0, 0.0, 0.0, -1.0, -0.5),
])
def test_create_model_rejects_bad_terms(loss, scale, l1, l2, lin, lo, hi):
    lib = pc.load()
    d, keep = _desc()
    b = np.zeros(4)
    mdl = _lib.pcdm_model(loss, 0, scale, l1, l2, lin, lo, hi)
    h = ctypes.c_void_p(1234)
    assert lib.pcdm_create_model(ctypes.byref(d), b.ctypes.data, ctypes.byref(mdl), 1, 0,
                                 ctypes.byref(h)) == _lib.PCDM_EINVAL
    assert h.value is None
    assert lib.pcdm_last_error()


@pytest.mark.parametrize("bp,tau", [
    ([0, 1, 2, 3], 0), ([0, 1, 2, 3], 4),     # tau outside [1, nblocks]
    ([1, 2, 3, 3], 1),                        # does not start at 0
    ([0, 1, 2, 2], 1),                        # empty block
    ([0, 2, 1, 3], 1),                        # decreasing
    ([0, 1, 2], 1),                           # ends before n (n = 3, two blocks cover 2 columns)
])
def test_create_group_rejects_bad_blocks(bp, tau):
    lib = pc.load()
    d, keep = _desc()
    b = np.zeros(4)
    bpa = np.array(bp, dtype=np.int64)
    h = ctypes.c_void_p(1234)
    st = lib.pcdm_create_group(ctypes.byref(d), b.ctypes.data, 0.1, bpa.ctypes.data, bpa.size - 1, tau, 0,
                               ctypes.byref(h))
    assert st == _lib.PCDM_EINVAL
    assert h.value is None


def test_create_group_rejects_blocks_over_sixteen_columns():
    lib = pc.load()
    n = 20
    cp = np.arange(n + 1, dtype=np.int64)
    ri = np.zeros(n, dtype=np.int32)
    v = np.ones(n)
    d = _lib.pcdm_csc(4, n, n, cp.ctypes.data, ri.ctypes.data, v.ctypes.data, _lib.PCDM_F64, 0)
    bpa = np.array([0, 17, 20], dtype=np.int64)
    h = ctypes.c_void_p(1234)
    assert lib.pcdm_create_group(ctypes.byref(d), np.zeros(4).ctypes.data, 0.1, bpa.ctypes.data, 2, 1, 0,
                                 ctypes.byref(h)) == _lib.PCDM_EINVAL
    assert b"16" in lib.pcdm_last_error()


def test_calibration_library_rejects_bad_sizes():
    """The benchmark's random-read calibration kernel (separate library, not
    part of the boundary) is built and checks its sizes before launching."""
    from paper_1212_0873_amd import build as hipbuild
    lib = ctypes.CDLL(hipbuild.CALIB_LIB)
    f = lib.pcdm_calib_random_gather
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    fake = ctypes.c_void_p(16)  # never dereferenced: every case below fails its size check first
    assert f(None, 10, 10, 0, fake, None) == 1
    assert f(fake, 0, 10, 0, fake, None) == 1
    assert f(fake, 1 << 32, 10, 0, fake, None) == 1
    assert f(fake, 10, 0, 0, fake, None) == 1
    assert lib.pcdm_calib_reads_per_thread() == 20
    g = lib.pcdm_calib_random_atomic
    g.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p]
    g.restype = ctypes.c_int
    assert g(None, 10, 10, 0, None) == 1
    assert g(fake, 0, 10, 0, None) == 1
    assert g(fake, 10, -1, 0, None) == 1


def test_every_option_key_is_documented():
    """The keys pcdm_set_option accepts are exactly the keys its comment in
    include/pcdm.h documents."""
    src = open(os.path.join(ROOT, "paper_1212_0873_amd", "csrc", "pcdm.hip")).read()
    start = src.index("int pcdm_set_option(pcdm_problem *h, const char *key, double value)\n{")
    body = src[start:src.index("\n}\n", start)]
    accepted = set(re.findall(r'k == "([a-z_0-9]+)"', body))
    hdr = open(os.path.join(ROOT, "include", "pcdm.h")).read()
    end = hdr.index("int pcdm_set_option(pcdm_problem *h, const char *key, double value);")
    block = hdr[hdr.rindex("/*", 0, end):end]
    documented = set(re.findall(r'"([a-z_0-9]+)"', block))
    assert accepted == documented, (accepted - documented, documented - accepted)



def test_gap_check_schedule():
    """Host logic of Problem.solve's "auto" schedule: the interval keeps the
    last evaluation's cost near a tenth of the stepping time and balances
    evaluation cost against the expected overshoot, within [1, 16]."""
    from paper_1212_0873_amd.api import next_check_interval as nci
    assert nci(0.0002, 0.00164, 300) == 9     # sqrt(2 * 300 * 0.2 / 1.64) = 8.55
    assert nci(0.0002, 0.00164, 0) == 2       # share term alone
    assert nci(0.0063, 0.211, 22) == 1        # sqrt(1.31) rounds to 1
    assert nci(0.0063, 0.211, 200) == 3
    assert nci(0.2, 0.2, 10**6) == 16
    assert nci(0.200, 0.211) == 10        # a full pass over A costs about an epoch
    assert nci(0.0063, 0.211) == 1        # the bounded route near the solution
    assert nci(0.0, 0.2) == 1
    assert nci(5.0, 0.01) == 16           # capped
    assert nci(0.03, 0.1, share=0.5) == 1
    assert nci(0.031, 0.1, share=0.1) == 4
    assert nci(1.0, 0.0) == 1 and nci(float("nan"), 1.0) == 1 and nci(1.0, float("nan")) == 1
    # a falling gap caps the interval at 0.8 of the epochs its rate needs:
    # 5.2 -> 1.47e-3 over 10 epochs is 0.44 per epoch, 8.9 epochs to 1e-6
    assert nci(0.19, 0.211, 22, trend=((12, 5.2), (22, 1.47e-3)), target=1e-6) == 7
    assert nci(0.19, 0.211, 22, trend=((12, 1e-3), (22, 2e-3)), target=1e-6) == 10   # rising: no cap
    assert nci(0.19, 0.211, 22, trend=((12, 5.2), (22, 1.1e-6)), target=1e-6) == 1   # almost there
    with pytest.raises(ValueError):
        pc.Problem.solve(object.__new__(pc.Problem), check_every=0)
