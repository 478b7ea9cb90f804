"""GPU parity at the edges of the input domain (bit-exact against the oracle):
the largest dimension the library accepts, denormal coordinates, and leaf
sizes at or above the point count."""
import numpy as np
import pytest

import oracle
from paper_2201_08288_amd import synth
from tests.gpu_common import KEYS, RULES, assert_same_tree, gpu_tree, oracle_tree

pytestmark = pytest.mark.gpu

D_MAX = 4096  # largest d of kd_build


@pytest.mark.parametrize("rule,key", [("exact", "cyclic"), ("exact", "maxvar"),
                                      ("fourier", "maxvar"), ("subset", "cyclic")])
def test_max_dimension(rule, key):
    print(f"case d={D_MAX} rule={rule} key={key}", flush=True)
    x = synth.gmm(300, D_MAX, seed=41)
    kw = dict(leaf_size=4, num_subsets=3, split_rule=RULES[rule], key_rule=KEYS[key])
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


def test_batched_with_max_dimension():
    print("case batched d=4096 mix", flush=True)
    import torch

    from paper_2201_08288_amd import kdtree
    shapes = [(300, D_MAX), (5000, 1), (64, 2048), (9000, 3)]
    xs = [synth.uniform24(n, d, seed=n + d) for n, d in shapes]
    kw = dict(leaf_size=8, num_subsets=4)
    trees = kdtree.build_batched([torch.from_numpy(x).cuda() for x in xs], **kw)
    torch.cuda.synchronize()
    for x, t in zip(xs, trees):
        assert_same_tree(t.to_numpy(), oracle_tree(x, **kw), x)


def denormal_points(n, d, seed):
    """Coordinates from the whole fp32 subnormal range (both signs), zeros of
    both signs and a few tiny normal values."""
    rng = np.random.default_rng(seed)
    bits = rng.integers(1, 1 << 23, size=(d, n), dtype=np.uint32)
    bits |= (rng.random((d, n)) < 0.5).astype(np.uint32) << 31
    x = bits.view(np.float32).copy()
    x[:, ::17] = 0.0
    x[:, 5::23] = -0.0
    x[:, 3::29] = np.float32(2.0 ** -120)
    return x


@pytest.mark.parametrize("rule", ["exact", "fourier", "subset"])
@pytest.mark.parametrize("key", ["cyclic", "maxvar"])
def test_denormal_coordinates(rule, key):
    print(f"case denormals rule={rule} key={key}", flush=True)
    x = denormal_points(6000, 3, seed=5)
    kw = dict(leaf_size=16, num_subsets=5, split_rule=RULES[rule], key_rule=KEYS[key])
    assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)


@pytest.mark.parametrize("leaf", [4999, 5000, 1 << 20])
def test_leaf_size_at_or_above_n(leaf):
    print(f"case n=5000 leaf={leaf}", flush=True)
    x = synth.uniform24(5000, 2, seed=leaf % 97)
    kw = dict(leaf_size=leaf)
    g = gpu_tree(x, **kw)[1]
    o = oracle_tree(x, **kw)
    assert_same_tree(g, o, x)
    assert g["num_leaves"] == (1 if leaf >= 5000 else 2)


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_default_depth_cap(rule):
    """Exponentially spaced values: FOURIER peels about one point per level and
    meets the default depth cap (the levels past the likely depth run in the
    small tail launch shape); the tree equals the oracle's for every rule."""
    print(f"case depth cap rule={rule}", flush=True)
    x = np.stack([(2.0 ** np.arange(0, 120)).astype(np.float32),
                  np.linspace(-1, 1, 120, dtype=np.float32)])
    kw = dict(leaf_size=1, num_subsets=4, split_rule=rule)
    g = gpu_tree(x, **kw)[1]
    o = oracle.build_tree(x, **kw)
    assert_same_tree(g, o, x)


@pytest.mark.parametrize("sigma", [4.0, 8.0])
def test_deep_tree_work_in_tail_shape(sigma):
    """Log-normal keys with FOURIER at J = 2: splits far from the median make
    the tree several levels deeper than a balanced one (h = 14; sigma 4:
    depth h + 5; sigma 8: the default cap h + 10, with oversize leaves and
    cells of more than 4096 points down to depth 15), so the levels past the
    likely depth, launched in the small tail shape, still split cells; the
    tree equals the oracle's."""
    print(f"case deep tree sigma={sigma}", flush=True)
    rng = np.random.default_rng(5)
    x = np.exp(rng.normal(0.0, sigma, size=(1, 200_000))).astype(np.float32)
    kw = dict(leaf_size=16, num_subsets=4, split_rule=1, fourier_J=2)
    g = gpu_tree(x, **kw)[1]
    o = oracle.build_tree(x, **kw)
    assert o["depth"] >= 14 + 5
    assert_same_tree(g, o, x)
