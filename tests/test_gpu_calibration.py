"""The benchmark's calibration kernels (libpcdm_calib.so) touch exactly the
positions they document: each thread's output of the random-read kernel is
the sum of the 20 table entries its fmix32 chain picks, and the random-atomic
kernel adds 1 at each of those picks, both recomputed on the host."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _fmix32(h):
    h = np.uint32(h)
    h ^= h >> np.uint32(16)
    h = np.uint32((int(h) * 0x85EBCA6B) & 0xFFFFFFFF)
    h ^= h >> np.uint32(13)
    h = np.uint32((int(h) * 0xC2B2AE35) & 0xFFFFFFFF)
    h ^= h >> np.uint32(16)
    return h


def test_calibration_reads_the_documented_positions():
    import torch
    assert torch.cuda.is_available()
    from paper_1212_0873_amd import build as hipbuild
    lib = ctypes.CDLL(hipbuild.CALIB_LIB)
    f = lib.pcdm_calib_random_gather
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    reads = lib.pcdm_calib_reads_per_thread()
    rng = np.random.default_rng(0)
    for m, nthreads, salt in ((1000, 300, 7), (4099, 1000, 123456789)):
        # integer-valued table: the float32 sums are exact in any order
        table = rng.integers(-1000, 1000, m).astype(np.float32)
        tab = torch.from_numpy(table).cuda()
        out = torch.empty(nthreads, dtype=torch.float32, device="cuda")
        assert f(tab.data_ptr(), m, nthreads, salt, out.data_ptr(), None) == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        want = np.empty(nthreads, dtype=np.float64)
        for t in range(nthreads):
            h = _fmix32(np.uint32(t) ^ np.uint32(salt))
            acc = 0.0
            for q in range(reads):
                h = _fmix32(np.uint32((int(h) + q) & 0xFFFFFFFF))
                acc += float(table[int(h) % m])
            want[t] = acc
        np.testing.assert_array_equal(got.astype(np.float64), want)


def test_calibration_atomics_hit_the_documented_positions():
    import torch
    assert torch.cuda.is_available()
    from paper_1212_0873_amd import build as hipbuild
    lib = ctypes.CDLL(hipbuild.CALIB_LIB)
    f = lib.pcdm_calib_random_atomic
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p]
    f.restype = ctypes.c_int
    reads = lib.pcdm_calib_reads_per_thread()
    m, nthreads, salt = 997, 500, 42
    tab = torch.zeros(m, dtype=torch.float32, device="cuda")
    assert f(tab.data_ptr(), m, nthreads, salt, None) == 0
    torch.cuda.synchronize()
    want = np.zeros(m)
    for t in range(nthreads):
        h = _fmix32(np.uint32(t) ^ np.uint32(salt))
        for q in range(reads):
            h = _fmix32(np.uint32((int(h) + q) & 0xFFFFFFFF))
            want[int(h) % m] += 1.0
    np.testing.assert_array_equal(tab.cpu().numpy().astype(np.float64), want)
