"""Whole-tree pins of the oracle: brute force on tiny inputs, invariants on
larger ones, closed-form shapes, and the paper's reported accuracy panel."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2201_08288_amd import synth
from tests import brute
from tests.invariants import check_tree, depth_of_nodes, descend, keys_of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _compare_with_brute(x, L, key, rule, S=1, max_depth=64):
    kr = oracle.KEY_CYCLIC if key == "cyclic" else oracle.KEY_MAXVAR
    sr = {"exact": oracle.SPLIT_EXACT, "subset": oracle.SPLIT_SUBSET}[rule]
    t = oracle.build_tree(x, leaf_size=L, key_rule=kr, split_rule=sr, num_subsets=S,
                          max_depth=max_depth)
    assert t["status"] == 0
    nodes, perm = brute.build(x, L, key=key, rule=rule, S=S, max_depth=max_depth)
    assert t["num_nodes"] == len(nodes)
    assert np.array_equal(t["perm"], np.array(perm, dtype=np.uint32))
    for k, nd in enumerate(nodes):
        assert t["node_begin"][k] == nd["begin"] and t["node_end"][k] == nd["end"]
        assert t["node_child"][k] == nd["child"]
        if nd["child"] >= 0:
            assert t["node_dim"][k] == nd["dim"]
            mk = int(keys_of(np.array([[nd["split"]]], dtype=np.float32))[0, 0])
            s = int(t["node_split"][k])
            if nd["kind"] == "le":
                assert s in (mk, mk - 1) if rule == "subset" else s == mk
            else:
                assert s == mk - 1
    return t


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 33, 64, 100, 199])
@pytest.mark.parametrize("L", [1, 4, 7])
def test_exact_cyclic_matches_brute_force(n, L):
    x = synth.uniform24(n, 3, seed=n * 31 + L)
    _compare_with_brute(x, L, "cyclic", "exact")


@pytest.mark.parametrize("n", [20, 77, 150])
def test_exact_heavy_ties_matches_brute_force(n):
    rng = np.random.default_rng(n)
    x = rng.integers(0, 4, size=(2, n)).astype(np.float32)
    _compare_with_brute(x, 3, "cyclic", "exact")
    x[:] = 1.0  # all equal: unsplittable root
    t = _compare_with_brute(x, 3, "cyclic", "exact")
    assert t["num_nodes"] == 1 and t["unsplittable"] == 1 and t["oversize"] == 1


@pytest.mark.parametrize("n", [30, 90, 180])
def test_exact_maxvar_matches_brute_force(n):
    rng = np.random.default_rng(n + 1)
    x = (np.rint(rng.standard_normal((4, n)) * np.array([[0.3], [2.0], [1.0], [1.5]]) * 1024)
         / 1024).clip(-7.99, 7.99).astype(np.float32)
    _compare_with_brute(x, 5, "maxvar", "exact")


@pytest.mark.parametrize("n,S", [(50, 1), (120, 4), (199, 16), (64, 64)])
def test_subset_matches_brute_force(n, S):
    x = synth.gmm(n, 2, seed=n + S)
    _compare_with_brute(x, 3, "cyclic", "subset", S=S)


def test_subset_mean_lies_between_subset_medians():
    """The fp32-rounded weighted mean never leaves [min, max] of the subset
    medians, so the tie rule always sees a candidate inside the cell's range."""
    rng = np.random.default_rng(31)
    for trial in range(300):
        n = int(rng.integers(2, 400))
        S = int(rng.integers(1, 40))
        kind = trial % 3
        if kind == 0:
            vals = rng.standard_normal(n).astype(np.float32)
        elif kind == 1:
            vals = np.full(n, np.float32(rng.standard_normal() * 1e3), dtype=np.float32)
        else:
            vals = (rng.integers(0, 3, size=n) * np.float32(2.0) ** rng.integers(-20, 20)).astype(np.float32)
        x = vals[None, :]
        ok, dim, split, cand = oracle.cell_split(x, np.arange(n), split_rule=oracle.SPLIT_SUBSET,
                                                 num_subsets=S, leaf_size=1)
        meds = [brute.lower_median_value([float(v) for v in vals[(r * n) // S:((r + 1) * n) // S]])
                for r in range(S) if ((r + 1) * n) // S > (r * n) // S]
        lo, hi = keys_of(np.array([[min(meds), max(meds)]], dtype=np.float32))[0]
        assert lo <= cand <= hi


def test_subset_with_one_subset_is_exact():
    x = synth.gmm(3000, 3, seed=2)
    a = oracle.build_tree(x, leaf_size=16, split_rule=oracle.SPLIT_SUBSET, num_subsets=1)
    b = oracle.build_tree(x, leaf_size=16, split_rule=oracle.SPLIT_EXACT)
    for k in ("perm", "node_begin", "node_child", "node_split", "leaf_offsets"):
        assert np.array_equal(a[k], b[k])


def test_depth_cap_gives_fixed_depth_tree():
    # §4: a depth-D tree has 2^D cells of about |X|/2^D points each.
    x = synth.uniform24(3000, 3, seed=4)
    t = oracle.build_tree(x, leaf_size=1, max_depth=5)
    assert t["num_leaves"] == 32 and t["depth"] == 5
    sizes = np.diff(t["leaf_offsets"].astype(np.int64))
    assert sizes.min() >= 3000 // 32 and sizes.max() <= -(-3000 // 32)


@pytest.mark.parametrize("k,l", [(10, 3), (12, 5), (16, 5)])
def test_power_of_two_exact_tree_is_perfect(k, l):
    # distinct keys in every coordinate: every leaf holds 2^l points at depth k - l
    rng = np.random.default_rng(k)
    n = 1 << k
    x = np.stack([rng.permutation(n) for _ in range(3)]).astype(np.float32) / np.float32(n)
    t = oracle.build_tree(x, leaf_size=1 << l)
    sizes = np.diff(t["leaf_offsets"].astype(np.int64))
    dep = depth_of_nodes(t)
    assert (sizes == 1 << l).all()
    assert (dep[t["leaf_node"]] == k - l).all()
    assert t["num_leaves"] == 1 << (k - l) and t["num_nodes"] == (1 << (k - l + 1)) - 1
    assert t["point_levels"] == (k - l) * n


@pytest.mark.parametrize("rule", [oracle.SPLIT_EXACT, oracle.SPLIT_FOURIER, oracle.SPLIT_SUBSET])
@pytest.mark.parametrize("gen,key", [("uniform24", oracle.KEY_CYCLIC), ("gmm", oracle.KEY_CYCLIC),
                                     ("student_t_grid", oracle.KEY_MAXVAR)])
def test_invariants_all_rules(rule, gen, key):
    x = synth.generate(gen, 5000, 4, seed=17)
    pool = synth.dirichlet_pool(128, 8, seed=2) if gen == "student_t_grid" else None
    t = oracle.build_tree(x, leaf_size=20, split_rule=rule, key_rule=key, num_subsets=8,
                          pool=pool, seed=99)
    assert t["status"] == 0
    check_tree(x, t, 20)
    # (iii) every point descends to the leaf that holds it
    leaf_of_point = np.empty(5000, dtype=np.int64)
    for k in range(t["num_leaves"]):
        leaf_of_point[t["perm"][t["leaf_offsets"][k]:t["leaf_offsets"][k + 1]]] = k
    assert np.array_equal(descend(t, x), leaf_of_point)
    assert np.array_equal(oracle.query_leaf(t, x[:, :300]), leaf_of_point[:300])
    sizes = np.diff(t["leaf_offsets"].astype(np.int64))
    assert (sizes[sizes > 20].size == t["oversize"])


def test_exact_children_sizes_ceil_floor():
    x = synth.uniform24(4097, 2, seed=8)
    t = oracle.build_tree(x, leaf_size=10)
    ch = t["node_child"]
    sz = (t["node_end"] - t["node_begin"]).astype(np.int64)
    for k in np.nonzero(ch >= 0)[0]:
        assert sz[ch[k]] == (sz[k] + 1) // 2 and sz[ch[k] + 1] == sz[k] // 2


def test_capacity_and_nonfinite_status():
    x = synth.uniform24(1000, 2, seed=1)
    t = oracle.build_tree(x, leaf_size=4, node_capacity=50)
    assert t["status"] == oracle.ECAPACITY
    y = x.copy()
    y[1, 7] = np.nan
    assert oracle.build_tree(y, leaf_size=4)["status"] == oracle.ENONFINITE
    y[1, 7] = np.inf
    assert oracle.build_tree(y, leaf_size=4)["status"] == oracle.ENONFINITE


def test_nan_query_returns_sentinel():
    x = synth.uniform24(500, 2, seed=3)
    t = oracle.build_tree(x, leaf_size=8)
    q = np.array([[np.nan], [0.5]], dtype=np.float32)
    assert oracle.query_leaf(t, q)[0] == 0xFFFFFFFF


def test_fourier_leaf_spread_shrinks_with_J_and_panel_report():
    """Thm 3.6 and 3.7 (§3.2) with the balanced-tree bound of §4: the leaf
    counts of a FOURIER tree approach |X| / 2^D as J grows.  On the §5.1
    workload shape (trivariate normal, rho = 0.5, depth 6) the largest
    relative deviation must shrink from J = 4 to 15 to 60.

    The §5.1 panel (J = (3,5), i.e. J = 15: counts within 2^25.45..2^25.52
    of an ideal 2^25.48232 at N = 3e9) comes from the paper's global
    single-pass method, not this per-level rule, so it is printed beside the
    measured spread as context and not asserted."""
    with open(os.path.join(GOLDEN, "paper_accuracy_panel.json")) as f:
        g = json.load(f)
    n = 3 * (1 << 16)
    x = synth.corr_normal(n, 3, rho=g["rho"], seed=21)
    worst = {}
    for J in (4, g["J"], 60):
        t = oracle.build_tree(x, leaf_size=1, max_depth=g["depth"],
                              split_rule=oracle.SPLIT_FOURIER, fourier_J=J, num_subsets=16)
        assert t["num_leaves"] == 2 ** g["depth"]
        rel = np.diff(t["leaf_offsets"].astype(np.int64)) / (n / 2 ** g["depth"])
        assert abs(rel.sum() - 2 ** g["depth"]) < 1e-9
        worst[J] = float(np.abs(np.log2(rel)).max())
        if J == g["J"]:
            print(f"per-level FOURIER, J={J}, n={n}: leaf counts 2^{np.log2(rel.min()):+.3f}"
                  f" .. 2^{np.log2(rel.max()):+.3f} of ideal; paper (global method, N=3e9):"
                  f" 2^{g['observed_min_log2'] - g['ideal_log2']:+.3f}"
                  f" .. 2^{g['observed_max_log2'] - g['ideal_log2']:+.3f}")
    assert worst[4] > worst[g["J"]] > worst[60], worst


def test_partition_checker_detects_wrong_split():
    from paper_2201_08288_amd import synth
    x = synth.gmm(5000, 3, seed=11)
    t = oracle.build_tree(x, leaf_size=8)
    assert oracle.check_partition(x, t) == 0
    assert oracle.check_partition(x[:, t["perm"]], t, permuted=True) == 0
    internal = np.nonzero(t["node_child"] >= 0)[0]
    bad = dict(t)
    bad["node_split"] = t["node_split"].copy()
    k = internal[0]
    # move the root split below its left child's largest key
    keys = oracle.keys_of_floats(x[t["node_dim"][k], t["perm"][t["node_begin"][k]:t["node_end"][t["node_child"][k]]]])
    bad["node_split"][k] = np.uint32(int(keys.max()) - 1)
    assert oracle.check_partition(x, bad) > 0
    swapped = dict(t)
    swapped["perm"] = t["perm"].copy()
    mid = t["node_end"][t["node_child"][k]]
    swapped["perm"][[0, mid]] = swapped["perm"][[mid, 0]]
    assert oracle.check_partition(x, swapped) > 0


@pytest.mark.parametrize("rule,key,pool", [(0, 0, False), (2, 1, True), (1, 1, False),
                                           (2, 0, False)])
def test_sampled_node_recompute_matches_whole_build(rule, key, pool):
    """Recomputing each node's split from its own points (ascending original
    index, depth, rank among its level's cells) reproduces the whole build;
    this is the check used on trees too large to rebuild."""
    from paper_2201_08288_amd import synth
    from tests.gpu_common import check_sampled_nodes
    x = synth.student_t_grid(6000, 4, seed=3 + rule)
    S = 8
    pl = synth.dirichlet_pool(32, S, seed=5) if pool else None
    kw = dict(num_subsets=S, key_rule=key, split_rule=rule, pool=pl, seed=9)
    t = oracle.build_tree(x, leaf_size=16, **kw)
    shift = oracle.maxvar_shift(x) if key == 1 else 0
    n = check_sampled_nodes(x, t, range(t["num_nodes"]), 16, shift=shift, **kw)
    assert n > 100
    # a wrong rank must be caught by the pool rule
    if pool:
        t2 = dict(t)
        t2["node_split"] = t["node_split"].copy()
        k = np.nonzero(t["node_child"] >= 0)[0][5]
        t2["node_split"][k] ^= np.uint32(1 << 20)
        with pytest.raises(AssertionError):
            check_sampled_nodes(x, t2, [k], 16, shift=shift, **kw)


@pytest.mark.parametrize("rule,key,pool", [(0, 1, True), (1, 0, False), (2, 1, True),
                                           (1, 1, True)])
def test_results_do_not_depend_on_thread_count(rule, key, pool):
    """The OpenMP oracle shares out cells, trees, coordinates and subsets;
    every tree must be the same bit for bit with one thread and with many
    (cells large enough that work inside a cell is shared too)."""
    x = synth.student_t_grid(300000, 5, seed=31 + rule)
    S = 16
    pl = synth.dirichlet_pool(64, S, seed=2) if pool else None
    kw = dict(leaf_size=40, num_subsets=S, key_rule=key, split_rule=rule, pool=pl, seed=4)
    prev = oracle.set_threads(1)
    try:
        one = oracle.build_tree(x, **kw)
    finally:
        oracle.set_threads(prev)
    many = oracle.build_tree(x, **kw)
    for k, v in one.items():
        assert np.array_equal(np.asarray(v), np.asarray(many[k])), k


def test_batched_oracle_equals_single_builds():
    shapes = [(1000, 2), (5000, 3), (70000, 8), (33, 4), (200000, 2)]
    xs = [synth.uniform24(n, d, seed=50 + i) for i, (n, d) in enumerate(shapes)]
    kw = dict(leaf_size=32, num_subsets=8, split_rule=oracle.SPLIT_FOURIER)
    batch = oracle.build_trees(xs, **kw)
    for x, b in zip(xs, batch):
        a = oracle.build_tree(x, **kw)
        for k, v in a.items():
            assert np.array_equal(np.asarray(v), np.asarray(b[k])), k


def test_default_depth_cap():
    """max_depth = 0 caps the depth at h + 10 (h: depth of a balanced tree,
    leaf_size * 2^h >= n); cells at the cap stay leaves and are counted as
    oversize.  FOURIER on exponentially spaced values peels about one point
    per level, so it meets the cap; EXACT on the same values does not."""
    x = (2.0 ** np.arange(0, 120)).astype(np.float32)[None, :]
    t = oracle.build_tree(x, leaf_size=1, split_rule=oracle.SPLIT_FOURIER)
    assert t["depth"] == 7 + 10 and t["oversize"] > 0
    deep = oracle.build_tree(x, leaf_size=1, split_rule=oracle.SPLIT_FOURIER, max_depth=64)
    assert deep["depth"] > 17 and deep["oversize"] == 0
    t = oracle.build_tree(x, leaf_size=1, split_rule=oracle.SPLIT_EXACT)
    assert t["depth"] == 7 and t["oversize"] == 0
