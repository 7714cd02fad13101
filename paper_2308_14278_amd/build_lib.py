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


# (scheme, precision) pairs the shooting kernels are instantiated for, one
# compilation of lm_shoot_inst.hip each
PAIRS = ((0, 0), (0, 1), (1, 0), (1, 1), (1, 2), (1, 4))


def build(verbose: bool = False, jobs: int | None = None) -> str:
    from concurrent.futures import ThreadPoolExecutor
    cc = hipcc()
    arch = ["--offload-arch=" + ARCH]
    with tempfile.TemporaryDirectory() as tmp:
        steps = []
        for name in ("lm_kernels", "lm_peak", "lm_analysis"):
            o = os.path.join(tmp, name + ".o")
            steps.append((o, [cc, *arch, *COMMON, "-c", os.path.join(CSRC, name + ".hip"),
                              "-o", o]))
        for s_, p_ in PAIRS:
            o = os.path.join(tmp, "lm_shoot_s%dp%d.o" % (s_, p_))
            steps.append((o, [cc, *arch, *COMMON, "-DLM_S=%d" % s_, "-DLM_PR=%d" % p_, "-c",
                              os.path.join(CSRC, "lm_shoot_inst.hip"), "-o", o]))
        # host-only C++: plain g++ against the HIP runtime headers
        ao = os.path.join(tmp, "lm_api.o")
        steps.append((ao, ["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
                           "-I" + os.path.join(ROCM, "include"), "-c",
                           os.path.join(CSRC, "lm_api.cpp"), "-o", ao]))
        n = jobs or min(len(steps), max(1, os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=n) as ex:
            list(ex.map(lambda st: _run(st[1]), steps))
        out = LIB + ".tmp%d" % os.getpid()
        _run([cc, *arch, "-shared", "-fPIC", "-o", out, *[o for o, _ in steps]])
        os.replace(out, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
