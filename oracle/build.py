"""Compile the plain-C FP64 oracle into ``oracle/libmdf_oracle.so``.

Test infrastructure only (see ``mdf_oracle.c``).  ``-ffp-contract=off`` keeps
the arithmetic exactly as written (no fused multiply-add contraction), so the
oracle's rounding does not depend on the host CPU.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mdf_oracle.c")
LIB = os.path.join(HERE, "libmdf_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True), file=sys.stderr)
