"""Compile the oracle's C source into oracle/liborc_pdhg.so with gcc.

Plain FP64, -O2, no FMA contraction and no fast-math, so every operation is
the IEEE binary64 operation the source writes.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdhg_oracle.c")
LIB = os.path.join(HERE, "liborc_pdhg.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-D_POSIX_C_SOURCE=199309L", "-Wall", "-Wextra", "-shared", "-fPIC",
           "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
