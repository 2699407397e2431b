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


SAN_LIB = os.path.join(HERE, "librewl_oracle_san.so")


def build_oracle(force=False, sanitize=False):
    """Build the oracle; with sanitize=True an AddressSanitizer +
    UndefinedBehaviorSanitizer build goes to librewl_oracle_san.so (load it
    with REWL_ORACLE_LIB set to that path and libasan preloaded)."""
    lib = SAN_LIB if sanitize else LIB
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(SRC):
        return lib
    tmp = lib + ".tmp"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-g"] if sanitize else []
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall"] + san + [
           "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    import sys
    print(build_oracle(force=True, sanitize="--sanitize" in sys.argv))
