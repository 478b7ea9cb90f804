"""GPU parity of FOURIER and SUBSET splits, the largest-variance key, pool
subsets and batched builds against the oracle (bit-exact)."""
import numpy as np
import pytest

import oracle
from paper_2201_08288_amd import synth
from tests.gpu_common import assert_same_tree, gpu_tree, oracle_tree

pytestmark = pytest.mark.gpu

FOURIER, SUBSET, EXACT = 1, 2, 0
MAXVAR = 1


@pytest.mark.parametrize("n", [1, 2, 33, 4095, 4097, 9000, 40000])
@pytest.mark.parametrize("J", [15, 40])
def test_fourier_sizes(n, J):
    print(f"case fourier n={n} J={J}", flush=True)
    x = synth.gmm(n, 3, seed=n + J)
    kw = dict(leaf_size=8, split_rule=FOURIER, fourier_J=J, num_subsets=16)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("J", [1, 2, 16, 17, 64])
def test_fourier_harmonic_counts(J):
    print(f"case fourier J={J}", flush=True)
    x = synth.uniform24(20000, 2, seed=J)
    kw = dict(leaf_size=16, split_rule=FOURIER, fourier_J=J)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("vals", [2, 7, 300])
def test_fourier_ties(vals):
    print(f"case fourier ties={vals}", flush=True)
    rng = np.random.default_rng(vals)
    x = (rng.integers(0, vals, size=(2, 25000)) * 0.37 - 4.0).astype(np.float32)
    kw = dict(leaf_size=16, split_rule=FOURIER)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


def test_fourier_wide_range_values():
    print("case fourier wide range", flush=True)
    rng = np.random.default_rng(5)
    x = (rng.standard_normal((3, 30000)) * 10.0 ** rng.integers(-30, 30, size=(3, 30000))).astype(
        np.float32)
    kw = dict(leaf_size=8, split_rule=FOURIER)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("n,S", [(100, 1), (5000, 7), (9000, 16), (40000, 256), (40000, 3),
                                 (65536, 4096)])
def test_subset_equal(n, S):
    print(f"case subset n={n} S={S}", flush=True)
    x = synth.gmm(n, 2, seed=S)
    kw = dict(leaf_size=8, split_rule=SUBSET, num_subsets=S)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("n,S", [(3 * 4097, 3), (2 * 8192 + 2, 2), (2 * 262145, 2),
                                 (5 * 262144 + 11, 5)])
def test_subset_large_segments(n, S):
    """Subsets just above 4096 points (two histogram workgroups each), at
    2 * 4096 + 1, and above 64 * 4096 (64 workgroups of more than 4096
    points each): every part of the block map against the oracle."""
    print(f"case subset large segments n={n} S={S}", flush=True)
    x = synth.uniform24(n, 2, seed=n)
    kw = dict(leaf_size=64, split_rule=SUBSET, num_subsets=S)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("n,S", [(3000, 8), (50000, 64)])
def test_subset_pool(n, S):
    print(f"case subset pool n={n} S={S}", flush=True)
    x = synth.student_t_grid(n, 3, seed=n)
    pool = synth.dirichlet_pool(512, S, alpha=0.5, seed=S)
    kw = dict(leaf_size=16, split_rule=SUBSET, num_subsets=S, pool=pool, seed=1234)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("rule", [EXACT, FOURIER, SUBSET])
@pytest.mark.parametrize("n", [3000, 40000])
def test_maxvar_key(rule, n):
    print(f"case maxvar rule={rule} n={n}", flush=True)
    x = synth.student_t_grid(n, 5, seed=n + rule)
    x *= np.array([[0.5], [3.0], [1.0], [2.0], [0.25]], dtype=np.float32)
    pool = synth.dirichlet_pool(64, 16, seed=3)
    kw = dict(leaf_size=32, key_rule=MAXVAR, split_rule=rule, num_subsets=16, pool=pool, seed=7)
    g = gpu_tree(x, **kw)[1]
    o = oracle_tree(x, **kw)
    assert len(set(o["node_dim"][o["node_child"] >= 0].tolist())) > 1
    assert_same_tree(g, o, x)


@pytest.mark.parametrize("scale", [1e-30, 1e-3, 7.0, 3e4])
def test_maxvar_grid_scales(scale):
    print(f"case maxvar scale={scale}", flush=True)
    x = (synth.gmm(20000, 4, seed=2) * np.float32(scale)).astype(np.float32)
    kw = dict(leaf_size=16, key_rule=MAXVAR)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("rule", [EXACT, FOURIER, SUBSET])
def test_plain_config_all_rules(rule):
    """The plain workload (n = 65,536, d = 3, S = 16, leaf 32) under each rule."""
    print(f"case plain config rule={rule}", flush=True)
    w = synth.WORKLOADS["plain_n65536_d3"]
    x = synth.generate(w["gen"], w["n"], w["d"])
    kw = dict(leaf_size=w["leaf_size"], num_subsets=w["num_subsets"], split_rule=rule)
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("rule", [EXACT, FOURIER, SUBSET])
def test_batched_equals_plain_and_oracle(rule):
    print(f"case batched rule={rule}", flush=True)
    import torch

    from paper_2201_08288_amd import kdtree
    shapes = [(1, 2), (5, 3), (700, 2), (4097, 3), (20000, 8), (33, 1), (9000, 32), (50000, 3)]
    xs = [synth.uniform24(n, d, seed=7 * n + d) for n, d in shapes]
    kw = dict(leaf_size=16, num_subsets=8, split_rule=rule)
    trees = kdtree.build_batched([torch.from_numpy(x).cuda() for x in xs], **kw)
    torch.cuda.synchronize()
    for x, t in zip(xs, trees):
        g = t.to_numpy()
        assert_same_tree(g, oracle_tree(x, **kw), x)
        p = gpu_tree(x, **kw)[1]
        assert_same_tree(g, p, x)


def test_batched_maxvar_pool_mixed():
    print("case batched maxvar pool", flush=True)
    import torch

    from paper_2201_08288_amd import kdtree
    shapes = [(3000, 4), (12000, 2), (100, 6), (45000, 3)]
    xs = [synth.student_t_grid(n, d, seed=n) for n, d in shapes]
    pool = synth.dirichlet_pool(128, 8, seed=9)
    kw = dict(leaf_size=20, num_subsets=8, split_rule=SUBSET, key_rule=MAXVAR, seed=99)
    trees = kdtree.build_batched([torch.from_numpy(x).cuda() for x in xs],
                                 subset_pool=torch.from_numpy(pool.view(np.int32)).cuda(), **kw)
    torch.cuda.synchronize()
    for x, t in zip(xs, trees):
        assert_same_tree(t.to_numpy(), oracle_tree(x, pool=pool, **kw), x)


@pytest.mark.parametrize("rule,key,pool", [(0, 0, False), (1, 0, False), (2, 0, False),
                                           (0, 1, True), (1, 1, True), (2, 1, True)])
def test_level_by_level_flag_same_tree(rule, key, pool):
    """KD_FLAG_LEVEL_BY_LEVEL sends small cells through one level per pass
    (every level streams through device memory); the tree is the oracle's,
    as with the on-chip completion of small cells."""
    from paper_2201_08288_amd import kdtree
    print(f"case level-by-level rule={rule} key={key} pool={pool}", flush=True)
    x = synth.student_t_grid(200_000, 6, seed=80 + rule + 3 * key)
    S = 16
    pl = synth.dirichlet_pool(64, S, seed=3) if pool else None
    kw = dict(leaf_size=24, num_subsets=S, split_rule=rule, key_rule=key, seed=5)
    g = gpu_tree(x, pool=pl, flags=kdtree.FLAG_LEVEL_BY_LEVEL, **kw)[1]
    assert_same_tree(g, oracle.build_tree(x, pool=pl, **kw), x)
