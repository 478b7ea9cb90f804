"""Host AddressSanitizer and UndefinedBehaviorSanitizer runs (CPU only):
the oracle builds trees for every rule, key and subset kind, and the C ABI's
host-side paths (bounds, argument checks, launch-shape setting, status
strings) run without a GPU.  Sanitizers instrument host code only."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.strip().endswith("ok")


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-fopenmp", "-ffp-contract=off", *SAN,
                           "-o", exe, os.path.join(ROOT, "oracle", "kd_oracle.c"),
                           os.path.join(HERE, "oracle_driver.c"), "-lm"])
    _run(exe)


def test_c_abi_host_paths_under_sanitizers(tmp_path):
    """The library's host code built with the sanitizers on the host side
    only; the device code is compiled as usual.  No GPU is touched."""
    from paper_2201_08288_amd import _build
    exe = str(tmp_path / "cabi_san")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]
    flags = [f for f in _build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    lib_obj, drv_obj = str(tmp_path / "kdtree.o"), str(tmp_path / "driver.o")
    subprocess.check_call(["/opt/rocm/bin/hipcc", *flags, *host_san, "-I", _build.INCLUDE, "-c",
                           "-o", lib_obj, _build.SRC])
    subprocess.check_call(["gcc", "-O1", *SAN, "-I", _build.INCLUDE, "-c", "-o", drv_obj,
                           os.path.join(HERE, "cabi_driver.c")])
    subprocess.check_call(["/opt/rocm/bin/hipcc", *flags, *host_san, "-o", exe, lib_obj, drv_obj])
    _run(exe)
