"""The gfx950 code object inside the built liblensmap.so: kernel resource
metadata (registers, LDS, spills) and a hash of its machine code.

The hash covers the code object's .text only: it is stable across rebuilds of
the same source (symbol names carry a per-build id) and changes exactly when
the generated code changes, so measurements of a kernel (HBM traffic counters)
can be tied to the code they were taken on.
"""
from __future__ import annotations

import hashlib
import os
import re
import shutil
import subprocess
import tempfile

from . import lensmap

LLVM = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin")
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def tools_available() -> bool:
    return all(os.path.exists(os.path.join(LLVM, t))
               for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf"))


def _extract(lib: str, tmp: str) -> str:
    """Unbundle the gfx950 code object of the library's kernels into tmp."""
    fat, co = os.path.join(tmp, "fatbin"), os.path.join(tmp, "gfx950.co")
    src = os.path.join(tmp, "lib.so")
    shutil.copy(lib, src)
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".hip_fatbin=" + fat,
                    src, os.path.join(tmp, "stripped.so")], check=True, capture_output=True)
    subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--type=o",
                    "--targets=" + TARGET, "--input=" + fat, "--output=" + co, "--unbundle"],
                   check=True, capture_output=True)
    return co


def kernel_metadata(lib: str = lensmap.LIB_PATH) -> dict:
    """{kernel symbol: {metadata key: value string}} from the code object notes."""
    with tempfile.TemporaryDirectory() as tmp:
        co = _extract(lib, tmp)
        notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", co], check=True,
                               capture_output=True, text=True).stdout
    kernels, cur = {}, {}
    for line in notes.splitlines():
        m = re.match(r"\s+-?\s*\.(\w+):\s+(\S+)\s*$", line)
        if not m:
            continue
        key, val = m.groups()
        if key == "agpr_count" and cur:  # first key of each kernel's record
            kernels[cur.get("name", "")] = cur
            cur = {}
        cur[key] = val
    if cur:
        kernels[cur.get("name", "")] = cur
    return kernels


def code_sha(lib: str = lensmap.LIB_PATH) -> str | None:
    """sha256[:16] of the code object's .text, or None without the tools."""
    if not tools_available() or not os.path.exists(lib):
        return None
    with tempfile.TemporaryDirectory() as tmp:
        co = _extract(lib, tmp)
        text = os.path.join(tmp, "text.bin")
        subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".text=" + text, co,
                        os.path.join(tmp, "co2.o")], check=True, capture_output=True)
        with open(text, "rb") as f:
            return hashlib.sha256(f.read()).hexdigest()[:16]
