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


def source_digest() -> str:
    """SHA-256 (first 16 hex digits) over the kernel sources and the compiler
    flags: identifies the code that a stored profile measured."""
    import hashlib
    h = hashlib.sha256()
    for d in DEPS:
        with open(d, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(flags()).encode())
    return h.hexdigest()[:16]


def build(force: bool = True, extra=(), out: str | None = None) -> str:
    out = out or LIB
    if not force and os.path.exists(out) and all(os.path.getmtime(out) >= os.path.getmtime(d) for d in DEPS):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = [hipcc(), *flags(extra), SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
