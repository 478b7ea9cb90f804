"""Pins of the oracle's building blocks against library routines, published
values and closed forms (CPU only)."""
import math
import struct

import numpy as np
import pytest

import oracle
from tests import brute


def _f32(x):
    return struct.unpack("<I", struct.pack("<f", x))[0]


# ---------------------------------------------------------------- encoding

def test_key_order_matches_float_order():
    rng = np.random.default_rng(1)
    specials = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-45, 1.17549435e-38,
                         -1.17549435e-38, 3.4028235e38, -3.4028235e38, 1.0, -1.0],
                        dtype=np.float32)
    x = np.concatenate([specials, rng.standard_normal(500).astype(np.float32),
                        (rng.standard_normal(200) * 1e-40).astype(np.float32)])
    keys = oracle.keys_of_floats(x)
    for i in range(0, x.size, 7):
        for j in range(0, x.size, 5):
            assert (keys[i] < keys[j]) == (x[i] < x[j])
            assert (keys[i] == keys[j]) == (x[i] == x[j])


def test_key_roundtrip_and_signed_zero():
    assert oracle.key_of_bits(_f32(-0.0)) == oracle.key_of_bits(_f32(0.0))
    for v in [1.5, -2.25, 1e-40, -3e38, float("inf"), float("-inf")]:
        b = _f32(v)
        assert oracle.bits_of_key(oracle.key_of_bits(b)) == b
    assert oracle.bits_of_key(oracle.key_of_bits(_f32(-0.0))) == _f32(0.0)


# ---------------------------------------------------------------- splitmix64

def test_splitmix64_published_sequence():
    # The reference SplitMix64 generator started from state 0 emits
    # 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4, 0x06c45d188009454f; output k is
    # the mix of state (k+1) * 0x9e3779b97f4a7c15.
    g = 0x9E3779B97F4A7C15
    assert oracle.splitmix64(0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(g) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64((2 * g) & (2**64 - 1)) == 0x06C45D188009454F


# ---------------------------------------------------------------- median

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 17, 63, 64, 65, 101, 4099, 200003])
def test_lower_median_against_numpy_sort(n):
    rng = np.random.default_rng(n)
    for trial in range(5):
        keys = rng.integers(0, 8 if trial % 2 else 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        assert oracle.lower_median(keys) == np.sort(keys)[(n - 1) // 2]
        assert oracle.lower_median(keys) == np.partition(keys, (n - 1) // 2)[(n - 1) // 2]


# ---------------------------------------------------------------- tie rule

def test_tie_rule_against_candidate_enumeration():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        n = int(rng.integers(1, 40))
        vals = sorted(int(v) for v in rng.integers(0, 6, size=n))
        m = int(rng.integers(min(vals), max(vals) + 1))
        lt = sum(v < m for v in vals)
        le = sum(v <= m for v in vals)
        ok, split = oracle.tie_rule(n, lt, le, m + 100)
        ref = brute.choose_split([float(v) for v in vals], float(m))
        if ref is None:
            assert not ok
            continue
        assert ok
        kind, nl = ref
        # the partition is the closest-to-balanced valid one ...
        assert sum(v + 100 <= split for v in vals) == nl
        # ... and the stored split is m ("u <= m") or m - 1 ("u < m"); when no
        # key equals m both describe the same partition
        if lt != le:
            assert split == (m + 100 if kind == "le" else m + 99)
        else:
            assert split in (m + 100, m + 99)


def test_tie_rule_distinct_keys_gives_ceil_half():
    for n in range(2, 50):
        k = (n - 1) // 2
        ok, split = oracle.tie_rule(n, k, k + 1, 1000)
        assert ok and split == 1000
        assert k + 1 == (n + 1) // 2


# ---------------------------------------------------------------- subsets

@pytest.mark.parametrize("n,S", [(10, 3), (65536, 16), (129, 256), (7, 1), (1000, 64)])
def test_equal_subsets_partition_cell(n, S):
    b = oracle.subset_bounds(n, S)
    assert b[0] == 0 and b[-1] == n
    sizes = np.diff(b.astype(np.int64))
    assert (sizes >= 0).all() and sizes.sum() == n
    assert set(sizes.tolist()) <= {n // S, -(-n // S)}


def test_pool_subsets_partition_cell():
    from paper_2201_08288_amd import synth
    pool = synth.dirichlet_pool(64, 16, alpha=0.5, seed=3)
    seen = set()
    for rank in range(200):
        b = oracle.subset_bounds(5000, 16, pool, seed=11, depth=3, rank=rank)
        assert b[0] == 0 and b[-1] == 5000
        assert (np.diff(b.astype(np.int64)) >= 0).all()
        row = oracle.splitmix64(11 ^ (3 << 32) ^ rank) % 64
        expect = np.concatenate([[0], (5000 * pool[row, 1:].astype(np.uint64)) >> np.uint64(32), [5000]])
        expect = np.maximum.accumulate(expect.astype(np.int64))
        assert (b.astype(np.int64) == expect).all()
        seen.add(tuple(b.tolist()))
    assert len(seen) > 20  # the hash visits many pool rows


# ---------------------------------------------------------------- max variance

def test_maxvar_shift_bounds_max_abs():
    rng = np.random.default_rng(0)
    for scale in [1e-3, 0.7, 1.0, 5.0, 4096.0]:
        x = (rng.standard_normal((3, 100)) * scale).astype(np.float32)
        s = oracle.maxvar_shift(x)
        E = 30 - s
        mx = float(np.abs(x.astype(np.float64)).max())
        assert 2.0 ** (E - 1) <= mx < 2.0 ** E
        assert E == math.frexp(mx)[1]


def test_maxvar_key_against_exact_rational_variance():
    rng = np.random.default_rng(5)
    for trial in range(30):
        d = int(rng.integers(2, 6))
        n = int(rng.integers(2, 60))
        # values on a 2^-10 grid with |x| < 8: the fixed-point grid is exact
        x = (np.rint(rng.standard_normal((d, n)) * rng.uniform(0.1, 2.0, size=(d, 1)) * 1024)
             / 1024).clip(-7.99, 7.99).astype(np.float32)
        idx = np.arange(n)
        shift = oracle.maxvar_shift(x)
        assert oracle.maxvar_key(x, idx, shift) == brute.exact_variance_key(x, idx)


def test_maxvar_key_numpy_var_when_clear_and_order_free():
    rng = np.random.default_rng(9)
    x = (rng.standard_normal((5, 400)) * np.array([[1.0], [3.0], [2.0], [0.5], [2.9]])).astype(np.float32)
    v = x.astype(np.float64).var(axis=1)
    top2 = np.sort(v)[-2:]
    assert top2[1] > 1.01 * top2[0]
    shift = oracle.maxvar_shift(x)
    idx = np.arange(400)
    k = oracle.maxvar_key(x, idx, shift)
    assert k == int(np.argmax(v))
    assert oracle.maxvar_key(x, rng.permutation(idx), shift) == k


def test_maxvar_ties_go_to_lowest_coordinate():
    x = np.array([[0, 1, 2, 3], [3, 2, 1, 0], [0, 0, 0, 0]], dtype=np.float32)
    shift = oracle.maxvar_shift(x)
    assert oracle.maxvar_key(x, np.arange(4), shift) == 0


# ---------------------------------------------------------------- sin / cos

def test_own_sincos_f32_within_ulps_of_libm():
    for x in np.linspace(0.0, 2.0, 2001, dtype=np.float32):
        s, c = oracle.sincos_f32(float(x))
        assert abs(s - math.sin(float(x))) <= 3e-7 * max(1.0, abs(math.sin(float(x))))
        assert abs(c - math.cos(float(x))) <= 3e-7


def test_own_sincos_f64_within_ulps_of_libm():
    for x in np.linspace(0.0, 2.0, 2001):
        s, c = oracle.sincos_f64(float(x))
        assert abs(s - math.sin(x)) <= 4.5e-16
        assert abs(c - math.cos(x)) <= 4.5e-16
    assert oracle.sincos_f64(0.0) == (0.0, 1.0)
    assert oracle.sincos_f32(0.0) == (0.0, 1.0)
