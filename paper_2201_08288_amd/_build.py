"""Compile libkdtree.so for gfx950 with hipcc (in-tree, no JIT cache)."""
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "kdtree.hip")
LIB = os.path.join(PKG, "libkdtree.so")
INCLUDE = os.path.join(ROOT, "include")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every a*b+c in device code stays two rounded operations (bit-exact with the CPU)
    "-ffp-contract=off",
    # keep fp32 denormals; no packed-fp32 instructions
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def sources():
    csrc = os.path.join(PKG, "csrc")
    return [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))] + [
        os.path.join(INCLUDE, "kdtree.h")]


def build(verbose=False):
    cmd = ["/opt/rocm/bin/hipcc", *HIPCC_FLAGS, "-I", INCLUDE, "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    build(verbose=True)
