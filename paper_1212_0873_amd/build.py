"""Build step for the HIP library (gfx950).  Run by ``__graft_entry__.build()``."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpcdm.so")
# memory-system calibration kernels used by bench.py (not the method)
CALIB_LIB = os.path.join(HERE, "libpcdm_calib.so")
# host entry points to the incremental bound's constants, for the CPU tests
CHECK_LIB = os.path.join(HERE, "libpcdm_check.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no v_pk_*_f32 generated for ordinary float code.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]


def calib_sources():
    d = os.path.join(CSRC, "calib")
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith(".hip")]


def check_sources():
    d = os.path.join(CSRC, "check")
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith(".hip")]


def _compile(srcs, out, verbose):
    tmp = out + f".tmp{os.getpid()}"
    cmd = [HIPCC, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile every .hip source directly under csrc/ into libpcdm.so, the
    calibration kernels under csrc/calib/ into libpcdm_calib.so and the
    host checks under csrc/check/ into libpcdm_check.so (always rebuilds
    all three)."""
    _compile(sources(), LIB, verbose)
    _compile(calib_sources(), CALIB_LIB, verbose)
    _compile(check_sources(), CHECK_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
