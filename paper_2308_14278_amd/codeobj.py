"""The gfx950 code object inside the built liblensmap.so: kernel resource
metadata (registers, LDS, spills) and per-kernel hashes of the machine code.

A kernel's hash covers its function bytes only: it is stable across rebuilds
of the same source (symbol names carry a per-build id) and across changes to
other kernels, and changes exactly when that kernel's generated code changes,
so measurements of a kernel (HBM traffic counters) can be tied to the code
they were taken on.
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


_BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _extract(lib: str, tmp: str) -> list[str]:
    """Unbundle the gfx950 code objects of the library's kernels into tmp: the
    fat-binary section holds one bundle per compiled HIP source."""
    fat = os.path.join(tmp, "fatbin")
    src = os.path.join(tmp, "lib.so")
    shutil.copy(lib, src)
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".hip_fatbin=" + fat,
                    src, os.path.join(tmp, "stripped.so")], check=True, capture_output=True)
    data = open(fat, "rb").read()
    starts = [m.start() for m in re.finditer(re.escape(_BUNDLE_MAGIC), data)]
    out = []
    for k, a in enumerate(starts):
        b = starts[k + 1] if k + 1 < len(starts) else len(data)
        part, co = os.path.join(tmp, "bundle%d" % k), os.path.join(tmp, "gfx950_%d.co" % k)
        with open(part, "wb") as fh:
            fh.write(data[a:b])
        r = subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--type=o",
                            "--targets=" + TARGET, "--input=" + part, "--output=" + co,
                            "--unbundle"], capture_output=True)
        if r.returncode == 0 and os.path.getsize(co) > 0:
            out.append(co)
    return out


def kernel_metadata(lib: str = lensmap.LIB_PATH) -> dict:
    """{kernel symbol: {metadata key: value string}} from the code object notes."""
    kernels = {}
    with tempfile.TemporaryDirectory() as tmp:
        for co in _extract(lib, tmp):
            notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", co],
                                   check=True, capture_output=True, text=True).stdout
            cur = {}
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


def kernel_code_sha(symbol: str, lib: str = lensmap.LIB_PATH) -> str | None:
    """sha256[:16] of one kernel's machine code (its function bytes in .text),
    or None without the tools or the symbol.  Other kernels changing size or
    place leave it unchanged (branches are relative and the shooting kernels
    address no global data)."""
    if not tools_available() or not os.path.exists(lib):
        return None
    with tempfile.TemporaryDirectory() as tmp:
        readelf = os.path.join(LLVM, "llvm-readelf")
        for co in _extract(lib, tmp):
            syms = subprocess.run([readelf, "--symbols", co], check=True, capture_output=True,
                                  text=True).stdout
            addr = size = None
            for line in syms.splitlines():
                f = line.split()
                if len(f) >= 8 and f[-1] == symbol and f[3] == "FUNC":
                    addr, size = int(f[1], 16), int(f[2])
            if addr is None:
                continue
            secs = subprocess.run([readelf, "-S", "-W", co], check=True, capture_output=True,
                                  text=True).stdout
            text = None
            for line in secs.splitlines():
                m = re.search(r"\]\s+\.text\s+\S+\s+([0-9a-f]+)\s+([0-9a-f]+)\s+([0-9a-f]+)",
                              line)
                if m:
                    text = (int(m.group(1), 16), int(m.group(2), 16), int(m.group(3), 16))
            if text is None or not (text[0] <= addr and addr + size <= text[0] + text[2]):
                return None
            with open(co, "rb") as fh:
                fh.seek(text[1] + (addr - text[0]))
                return hashlib.sha256(fh.read(size)).hexdigest()[:16]
    return None
