"""The C ABI without a GPU: libkdtree.so loads, exports every function that
include/kdtree.h declares, and its host-only calls (sizes, parameter
checks, status strings) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kdtree.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(kd_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_08288_amd import _build
    if not os.path.exists(_build.LIB):
        _build.build()
    return ctypes.CDLL(_build.LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("kd_build", "kd_build_batched", "kd_query_leaf", "kd_tree_bounds",
              "kd_batch_bounds", "kd_build_profiled", "kd_status_string", "kd_version"):
        assert f in names, f


def test_library_exports_every_declared_function(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_host_only_calls(lib):
    from paper_2201_08288_amd import kdtree
    lib.kd_version.restype = ctypes.c_int
    assert lib.kd_version() >= 1
    lib.kd_status_string.restype = ctypes.c_char_p
    lib.kd_status_string.argtypes = [ctypes.c_int32]
    strings = {lib.kd_status_string(s) for s in range(7)}
    assert len(strings) == 7 and all(strings)
    L = kdtree.lib()
    cap, ws = ctypes.c_uint64(), ctypes.c_uint64()
    p = kdtree.make_params(leaf_size=32, num_subsets=16)
    assert L.kd_tree_bounds(65536, 3, ctypes.byref(p), ctypes.byref(cap), ctypes.byref(ws)) == 0
    assert cap.value == 4 * (65536 // 32) + 64 and ws.value > 0
    for bad in (dict(leaf_size=0), dict(num_subsets=0), dict(num_subsets=4097),
                dict(split_rule=3), dict(key_rule=2), dict(split_rule=1, fourier_J=0),
                dict(split_rule=1, fourier_J=65), dict(max_depth=129)):
        kw = dict(leaf_size=32, num_subsets=16)
        kw.update(bad)
        q = kdtree.make_params(**kw)
        assert L.kd_tree_bounds(1000, 3, ctypes.byref(q), ctypes.byref(cap),
                                ctypes.byref(ws)) == kdtree.KD_EINVAL, bad
    assert L.kd_tree_bounds(0, 3, ctypes.byref(p), ctypes.byref(cap), ctypes.byref(ws)) == \
        kdtree.KD_EINVAL
    assert L.kd_tree_bounds(10, 0, ctypes.byref(p), ctypes.byref(cap), ctypes.byref(ws)) == \
        kdtree.KD_EINVAL


def test_workspace_grows_with_size(lib):
    from paper_2201_08288_amd import kdtree
    p = kdtree.make_params(leaf_size=64, num_subsets=256)
    small = kdtree.tree_bounds(1 << 16, 8, p)[1]
    large = kdtree.tree_bounds(1 << 24, 8, p)[1]
    assert large > 100 * small
    # two working copies of the columns and permutation at least
    assert large >= 2 * (8 + 1) * 4 * (1 << 24)


def test_tuning_round_trip(lib):
    from paper_2201_08288_amd import kdtree
    before = kdtree.get_tuning()
    try:
        kdtree.set_tuning(hist_blocks=1024, scatter_blocks=2048, small_blocks=4096, digit_bits=8)
        assert kdtree.get_tuning() == {"hist_blocks": 1024, "scatter_blocks": 2048,
                                       "small_blocks": 4096, "digit_bits": 8}
        # only 11- and 8-bit digits exist; a rejected setting leaves the old one
        for bad in (1, 9, 10, 12, 16):
            t = kdtree.Tuning(0, 0, 0, bad)
            assert kdtree.lib().kd_set_tuning(ctypes.byref(t)) == kdtree.KD_EINVAL
        assert kdtree.get_tuning()["digit_bits"] == 8
    finally:
        kdtree.set_tuning(**before)
    assert kdtree.get_tuning() == before
    L = kdtree.lib()
    assert L.kd_set_tuning(None) == kdtree.KD_EINVAL and L.kd_get_tuning(None) == kdtree.KD_EINVAL


def test_query_and_global_argument_checks(lib):
    """Parameter errors are reported on the host, before any device work."""
    from paper_2201_08288_amd import kdtree
    L = kdtree.lib()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks come first
    t = kdtree.TreeStruct()
    for f in kdtree.KDTree.FIELDS:
        setattr(t, f, fake.value)
    t.hdr = fake.value
    t.points_out = fake.value
    t.node_capacity = 16
    E = kdtree.KD_EINVAL
    for k in (0, 65):
        assert L.kd_query_knn(ctypes.byref(t), 10, fake, 4, 2, 4, k, fake, fake, None) == E
    assert L.kd_query_knn(ctypes.byref(t), 10, fake, 4, 0, 4, 1, fake, fake, None) == E  # d = 0
    assert L.kd_query_knn(ctypes.byref(t), 10, fake, 4, 2, 3, 1, fake, fake, None) == E  # ldq < nq
    t.points_out = None
    assert L.kd_query_knn(ctypes.byref(t), 10, fake, 4, 2, 4, 1, fake, fake, None) == E
    assert L.kd_query_box(ctypes.byref(t), 10, fake, fake, 4, 2, 4, fake, None, None, None) == E
    t.points_out = fake.value
    assert L.kd_query_box(ctypes.byref(t), 10, fake, fake, 4, 2, 4, fake, None, fake, None) == E
    for p, J in ((0, 15), (4, 15), (3, 0), (3, 16)):
        assert L.kd_global_moments(fake, 100, p, 100, J, fake, None) == E, (p, J)
    assert L.kd_global_moments(fake, 0, 3, 100, 15, fake, None) == E
    assert L.kd_global_moments(fake, 100, 3, 99, 15, fake, None) == E
    for depth in (0, 13):
        assert L.kd_global_solve(fake, 3, 15, depth, fake, None) == E
        assert L.kd_global_counts(fake, 100, 3, 100, fake, depth, fake, None) == E
    assert L.kd_global_solve(None, 3, 15, 6, fake, None) == E
