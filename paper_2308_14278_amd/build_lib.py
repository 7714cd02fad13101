"""Build liblensmap.so (HIP for gfx950) in-tree: paper_2308_14278_amd/liblensmap.so.

Usage: python -m paper_2308_14278_amd.build_lib
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblensmap.so")
ARCH = os.environ.get("LENSMAP_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU ops.
# -ffp-contract=off: every FMA is written out, so the shooting kernel and the
# per-ray probes round identically.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory() as tmp:
        ko = os.path.join(tmp, "lm_kernels.o")
        ao = os.path.join(tmp, "lm_api.o")
        po = os.path.join(tmp, "lm_peak.o")
        _run([cc, "--offload-arch=" + ARCH, *COMMON, "-c",
              os.path.join(CSRC, "lm_kernels.hip"), "-o", ko])
        _run([cc, "--offload-arch=" + ARCH, *COMMON, "-c",
              os.path.join(CSRC, "lm_peak.hip"), "-o", po])
        yo = os.path.join(tmp, "lm_analysis.o")
        _run([cc, "--offload-arch=" + ARCH, *COMMON, "-c",
              os.path.join(CSRC, "lm_analysis.hip"), "-o", yo])
        # host-only C++: plain g++ against the HIP runtime headers
        _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
              "-I" + os.path.join(ROCM, "include"), "-c", os.path.join(CSRC, "lm_api.cpp"),
              "-o", ao])
        out = LIB + ".tmp%d" % os.getpid()
        _run([cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out, ko, po, yo, ao])
        os.replace(out, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
