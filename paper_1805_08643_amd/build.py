"""Build the HIP library ``libmrtlbm.so`` for gfx950, in-tree.

One translation unit (csrc/lbm_api.hip) holds the kernels and the C ABI.
Packed-FP32 instructions are disabled for the device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lbm_api.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "lbm_kernels.hpp"), os.path.join(HERE, "csrc", "lbm_device.hpp"),
        os.path.join(ROOT, "include", "mrt_lbm.h")]
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libmrtlbm.so")
# Data-movement probes of the HBM ceiling (include/mrt_probe.h), a library of
# their own so that the step library carries none of them.
PROBE_SRC = os.path.join(HERE, "csrc", "probe.hip")
PROBE_DEPS = [PROBE_SRC, os.path.join(ROOT, "include", "mrt_probe.h"), os.path.join(ROOT, "include", "mrt_lbm.h")]
PROBE_LIB = os.path.join(LIBDIR, "libmrtprobe.so")
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(extra=()):
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-ffp-contract=fast", "-munsafe-fp-atomics", "-Wall", *extra]


def code_text(src: str) -> str:
    """C/C++ source without its comments, with every run of blank space made
    one space: what the compiler sees of it.  String and character literals
    are kept as written."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":  # literal: copy up to the matching unescaped quote
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_digest() -> str:
    """SHA-256 (first 16 hex digits) over the code of the kernel sources
    (``code_text``: comments and layout do not count) and the compiler flags:
    identifies the code that a stored profile measured."""
    import hashlib
    h = hashlib.sha256()
    for d in DEPS:
        with open(d, encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    h.update(" ".join(flags()).encode())
    return h.hexdigest()[:16]


def _compile(src, deps, out, force, extra=()):
    if not force and os.path.exists(out) and all(os.path.getmtime(out) >= os.path.getmtime(d) for d in deps):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = [hipcc(), *flags(extra), src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True, extra=(), out: str | None = None) -> str:
    return _compile(SRC, DEPS, out or LIB, force, extra)


def build_probe(force: bool = True) -> str:
    return _compile(PROBE_SRC, PROBE_DEPS, PROBE_LIB, force)


if __name__ == "__main__":
    force = "--if-stale" not in sys.argv
    print(build(force=force))
    print(build_probe(force=force))
