"""Build the C oracle into ``oracle/liblbm_oracle.so`` (test infrastructure).

Plain gcc, FP64, ``-ffp-contract=off`` so that no fused multiply-add changes
the rounding of the written-out formulas, no fast-math, OpenMP over z-planes.

``build(defines=..., out=...)`` also builds variant libraries for the tests
(for example with a planted mistake, ``ORACLE_PLANT=<n>``) or with the host
sanitizers (``sanitize=True``) into a path of the caller's choice.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True, defines: dict | None = None, out: str | None = None) -> str:
    out = out or LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp"
    dflags = [f"-D{k}={v}" for k, v in (defines or {}).items()]
    cmd = ["gcc", *CFLAGS, *dflags, "-shared", "-fPIC", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
