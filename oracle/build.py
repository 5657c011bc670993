"""Compile the CPU oracle (test infrastructure) into ``oracle/libtsds_oracle.so``.

Plain gcc, ``-O2 -ffp-contract=off``: no fused multiply-add, so every floating
point expression in the oracle is rounded exactly as it is written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tsds_oracle.c")
LIB = os.path.join(HERE, "libtsds_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-Wall", "-Wextra", "-pthread", "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
