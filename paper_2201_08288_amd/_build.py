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
    # roctx ranges (build, level, kernel class) on the host timeline
    "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
]


def sources():
    csrc = os.path.join(PKG, "csrc")
    return [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))] + [
        os.path.join(INCLUDE, "kdtree.h")]


HASH = LIB + ".srchash"  # hash of the sources the library was built from


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in sources():
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose=False):
    cmd = ["/opt/rocm/bin/hipcc", *HIPCC_FLAGS, "-I", INCLUDE, "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    digest = source_hash()
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    with open(HASH, "w") as fh:
        fh.write(digest + "\n")
    return LIB


def stale():
    """True when the library is missing or was built from other sources."""
    if not os.path.exists(LIB) or not os.path.exists(HASH):
        return True
    with open(HASH) as fh:
        return fh.read().strip() != source_hash()


if __name__ == "__main__":
    build(verbose=True)
