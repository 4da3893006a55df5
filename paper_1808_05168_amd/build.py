"""Builds libfnlb.so (the HIP library behind include/fnlb.h) for gfx950.

Run as ``python -m paper_1808_05168_amd.build`` or call ``build()``.  The
library is built in-tree next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfnlb.so")
SOURCES = ["k_step.hip", "k_step2.hip", "k_observe.hip", "k_adjoint.hip", "fnlb_api.hip"]
HEADERS = ["fnlb_device.hpp", "fnlb_fft.hpp", "fnlb_internal.hpp", "fnlb_node.hpp",
           "fnlb_state.hpp"]
ARCH = os.environ.get("FNLB_OFFLOAD_ARCH", "gfx950")


def source_id() -> str:
    """Hash of every source the library is built from (kernels, runtime,
    internal headers, the C header and this build script), 16 hex digits.
    The build bakes it into the library (fnlb_build_id) and the binding
    compares it with the sources it finds, so a stale library is refused."""
    import hashlib
    h = hashlib.sha256()
    paths = [os.path.join(CSRC, n) for n in SOURCES + HEADERS]
    paths += [os.path.join(ROOT, "include", "fnlb.h"), os.path.abspath(__file__)]
    for p in paths:
        with open(p, "rb") as fh:
            h.update(os.path.basename(p).encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-shared",
           # keep packed FP32 instructions out of the device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           '-DFNLB_BUILD_ID="%s"' % source_id()]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
