"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (one kd_build over the whole resident input).

n = 2^24, d = 8 (Gaussian mixture, 256 equal subsets, leaf 64): the EXACT
tree is compared with the oracle's whole build element by element; FOURIER
and SUBSET trees are checked on sampled nodes, each recomputed by the oracle
from that node's own points, plus the partition property over every node.

n = 2^26, d = 16 (Student-t on a 2^-10 grid, Dirichlet(1/2) subset pool of
4096 rows x 64 subsets, largest-variance key, leaf 128): sampled nodes and
the full partition property, for every split rule.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2201_08288_amd import synth
from tests.gpu_common import assert_same_tree, check_sampled_nodes, gpu_tree

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def structural(x, g, leaf_size):
    """Every point in exactly one leaf, leaf ranges tile [0, n), the permuted
    points are the inputs in tree order, and no point lies on the wrong side
    of any split."""
    d, n = x.shape
    perm = g["perm"]
    assert np.array_equal(np.bincount(perm, minlength=n), np.ones(n, dtype=np.int64))
    lo = g["leaf_offsets"]
    assert lo[0] == 0 and lo[-1] == n and (np.diff(lo.astype(np.int64)) > 0).all()
    leaves = g["leaf_node"]
    assert np.array_equal(g["node_begin"][leaves], lo[:-1])
    assert np.array_equal(g["node_end"][leaves], lo[1:])
    from concurrent.futures import ThreadPoolExecutor

    def column(c):
        return np.array_equal(g["points_out"][c].view(np.uint32), x[c, perm].view(np.uint32))

    with ThreadPoolExecutor(max_workers=8) as ex:
        same = list(ex.map(column, range(d)))
    assert all(same), [c for c in range(d) if not same[c]]
    bad = oracle.check_partition(g["points_out"], g, permuted=True)
    assert bad == 0, bad
    size = (g["node_end"] - g["node_begin"]).astype(np.int64)
    over = int(((g["node_child"] < 0) & (size > leaf_size)).sum())
    assert over == g["oversize"], (over, g["oversize"])


def sample_nodes(g, rng, top_depth, count):
    from tests.gpu_common import node_depths
    dep = node_depths(g["node_child"])
    top = np.nonzero(dep <= top_depth)[0]
    rest = np.nonzero(dep > top_depth)[0]
    pick = rng.choice(rest, size=min(count, rest.size), replace=False)
    return np.concatenate([top, np.sort(pick)])


@pytest.fixture(scope="module")
def scale_input():
    w = synth.WORKLOADS["scale_n2^24_d8"]
    log("generating n=2^24 d=8 Gaussian mixture")
    return w, synth.generate(w["gen"], w["n"], w["d"])


@pytest.fixture(scope="module")
def hard_input():
    w = synth.WORKLOADS["hard_n2^26_d16"]
    log("generating n=2^26 d=16 Student-t grid")
    x = synth.generate(w["gen"], w["n"], w["d"])
    pool = synth.dirichlet_pool(w["pool_entries"], w["num_subsets"], w["pool_alpha"])
    return w, x, pool


def test_scale_exact_whole_tree(scale_input):
    w, x = scale_input
    kw = dict(leaf_size=w["leaf_size"], num_subsets=w["num_subsets"], split_rule=0)
    log("case scale exact: gpu build")
    _, g = gpu_tree(x, **kw)
    log(f"gpu header {[(k, g[k]) for k in ('num_nodes', 'num_leaves', 'depth', 'point_levels')]}")
    log("oracle whole build")
    o = oracle.build_tree(x, **kw)
    assert_same_tree(g, o, x)


@pytest.mark.parametrize("rule", [1, 2])
def test_scale_sampled(scale_input, rule):
    w, x = scale_input
    kw = dict(num_subsets=w["num_subsets"], split_rule=rule, fourier_J=15)
    log(f"case scale rule={rule}: gpu build")
    _, g = gpu_tree(x, leaf_size=w["leaf_size"], **kw)
    assert g["status"] == 0
    structural(x, g, w["leaf_size"])
    nodes = sample_nodes(g, np.random.default_rng(rule), 2, 40)
    log(f"checking {nodes.size} sampled nodes")
    assert check_sampled_nodes(x, g, nodes, w["leaf_size"], log=log, **kw) > 20


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_hard_sampled(hard_input, rule):
    w, x, pool = hard_input
    kw = dict(num_subsets=w["num_subsets"], split_rule=rule, key_rule=1, fourier_J=15,
              seed=w.get("seed", 0))
    log(f"case hard rule={rule}: gpu build")
    _, g = gpu_tree(x, leaf_size=w["leaf_size"], pool=pool, **kw)
    assert g["status"] == 0
    log(f"gpu header {[(k, g[k]) for k in ('num_nodes', 'num_leaves', 'depth', 'unsplittable')]}")
    structural(x, g, w["leaf_size"])
    shift = oracle.maxvar_shift(x)
    nodes = sample_nodes(g, np.random.default_rng(10 + rule), 1, 30)
    log(f"checking {nodes.size} sampled nodes")
    assert check_sampled_nodes(x, g, nodes, w["leaf_size"], shift=shift, pool=pool, log=log,
                               **kw) > 15
