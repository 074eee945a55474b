"""Compile the oracle's C source into oracle/liborc_pdhg.so with gcc.

Plain FP64, -O2, no FMA contraction and no fast-math, so every operation is
the IEEE binary64 operation the source writes.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdhg_oracle.c")
LIB = os.path.join(HERE, "liborc_pdhg.so")


def build(force: bool = True, mutation: int = 0, out: str | None = None) -> str:
    """Compile the oracle; `mutation` > 0 plants the numbered mistake (tests
    of the pins only) into the library written to `out`."""
    lib = out or LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-D_POSIX_C_SOURCE=199309L", f"-DORC_MUT={int(mutation)}", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
