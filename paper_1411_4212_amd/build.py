"""Build librewl.so (HIP kernels + C ABI) for gfx950, in-tree."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librewl.so")
SOURCES = ["rewl_kernels.hip", "rewl_mlp.hip", "rewl_api.cpp"]
HEADERS = ["rewl_device.h", "rewl_internal.h", "rewl_mlp_device.h"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # every floating-point operation exactly as written (no FMA contraction),
    # needed by the deterministic FP64 mode; fused forms are spelled out
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(force=True, verbose=False):
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [
        os.path.join(HERE, "..", "include", "rewl.h")]
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["hipcc"] + FLAGS + ["-x", "hip"] + sources() + ["-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
