"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C compiled by gcc with -ffp-contract=off and no fast-math,
so every floating-point operation is one IEEE binary64 operation in source
order.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rewl_oracle.c")
LIB = os.path.join(HERE, "librewl_oracle.so")


def build_oracle(force=False):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall",
           "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(force=True))
