"""GPU parity of the EXACT rule with cyclic keys against the oracle (bit-exact)."""
import numpy as np
import pytest

from paper_2201_08288_amd import synth
from tests.gpu_common import assert_same_tree, gpu_tree, oracle_tree

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 3, 31, 32, 33, 100, 4095, 4096, 4097, 8193, 12289, 40000])
@pytest.mark.parametrize("d", [1, 3])
def test_exact_sizes(n, d):
    print(f"case exact n={n} d={d}", flush=True)
    x = synth.uniform24(n, d, seed=n + 7 * d)
    kw = dict(leaf_size=8)
    g = gpu_tree(x, **kw)[1]
    assert_same_tree(g, oracle_tree(x, **kw), x)


@pytest.mark.parametrize("L", [1, 5, 32, 64])
def test_exact_leaf_sizes(L):
    print(f"case exact leaf={L}", flush=True)
    x = synth.gmm(20000, 4, seed=L)
    g = gpu_tree(x, leaf_size=L)[1]
    assert_same_tree(g, oracle_tree(x, leaf_size=L), x)


@pytest.mark.parametrize("vals", [2, 5, 1000])
def test_exact_heavy_ties(vals):
    print(f"case exact ties={vals}", flush=True)
    rng = np.random.default_rng(vals)
    x = rng.integers(0, vals, size=(3, 30000)).astype(np.float32)
    g = gpu_tree(x, leaf_size=16)[1]
    o = oracle_tree(x, leaf_size=16)
    assert_same_tree(g, o, x)


def test_exact_all_equal_and_signed_zero():
    print("case exact all-equal", flush=True)
    x = np.zeros((2, 9000), dtype=np.float32)
    x[0, ::2] = -0.0
    g = gpu_tree(x, leaf_size=4)[1]
    o = oracle_tree(x, leaf_size=4)
    assert o["unsplittable"] == 1 and o["num_nodes"] == 1
    assert_same_tree(g, o, x)


def test_exact_max_depth():
    print("case exact max_depth", flush=True)
    x = synth.uniform24(50000, 3, seed=3)
    g = gpu_tree(x, leaf_size=1, max_depth=6)[1]
    assert_same_tree(g, oracle_tree(x, leaf_size=1, max_depth=6), x)


def test_exact_plain_config():
    """The plain workload: n = 65,536, d = 3, 24-bit uniform, leaf size 32."""
    print("case exact plain config", flush=True)
    w = synth.WORKLOADS["plain_n65536_d3"]
    x = synth.generate(w["gen"], w["n"], w["d"])
    kw = dict(leaf_size=w["leaf_size"], num_subsets=w["num_subsets"])
    g = gpu_tree(x, **kw)[1]
    o = oracle_tree(x, **kw)
    assert o["num_leaves"] == 2048
    assert_same_tree(g, o, x)


def test_nonfinite_input_status():
    print("case exact nonfinite", flush=True)
    from paper_2201_08288_amd import kdtree
    x = synth.uniform24(5000, 2, seed=1)
    x[1, 17] = np.nan
    g = gpu_tree(x, leaf_size=8)[1]
    assert g["status"] == kdtree.KD_ENAN
    x[1, 17] = -np.inf
    assert gpu_tree(x, leaf_size=8)[1]["status"] == kdtree.KD_ENAN


def test_capacity_status():
    print("case exact capacity", flush=True)
    from paper_2201_08288_amd import kdtree
    x = synth.uniform24(5000, 2, seed=2)
    g = gpu_tree(x, leaf_size=4, node_capacity=100)[1]
    assert g["status"] == kdtree.KD_ECAPACITY


def test_query_leaf_matches_oracle_and_points():
    print("case query", flush=True)
    import torch

    from paper_2201_08288_amd import kdtree
    x = synth.gmm(30000, 3, seed=9)
    t, g = gpu_tree(x, leaf_size=16)
    o = oracle_tree(x, leaf_size=16)
    assert_same_tree(g, o, x)
    q = np.concatenate([x[:, ::7], synth.gmm(500, 3, seed=10)], axis=1)
    q[1, 3] = np.nan
    got = kdtree.query_leaf(t, torch.from_numpy(q).cuda()).cpu().numpy().view(np.uint32)
    import oracle
    assert np.array_equal(got, oracle.query_leaf(o, q))
    assert got[3] == 0xFFFFFFFF
    leaf_of_point = np.empty(x.shape[1], dtype=np.int64)
    for k in range(g["num_leaves"]):
        leaf_of_point[g["perm"][g["leaf_offsets"][k]:g["leaf_offsets"][k + 1]]] = k
    allq = kdtree.query_leaf(t, torch.from_numpy(x).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(allq.astype(np.int64), leaf_of_point)


def test_strided_input_and_no_points_out():
    print("case strided", flush=True)
    import torch

    from paper_2201_08288_amd import kdtree
    x = synth.uniform24(10000, 3, seed=4)
    big = torch.zeros((3, 10240), dtype=torch.float32)
    big[:, :10000] = torch.from_numpy(x)
    t = kdtree.build(big.cuda()[:, :10000], leaf_size=8, points_out=False)
    g = t.to_numpy()
    assert_same_tree(g, oracle_tree(x, leaf_size=8))


@pytest.mark.parametrize("rule,key", [(0, 0), (0, 1), (1, 1), (2, 0), (2, 1)])
def test_strided_large_root_every_rule(rule, key):
    """A root of more than 4096 points is split at level 0 straight from the
    caller's [d][ld] points (no working copy): ld > n, -0.0 and subnormal
    coordinates among them, every rule and key, with and without points_out."""
    import torch

    from paper_2201_08288_amd import kdtree
    print(f"case strided large root rule={rule} key={key}", flush=True)
    n, d, ld = 70001, 4, 70001 + 333
    x = synth.gmm(n, d, seed=40 + rule)
    x[1, ::13] = -0.0
    x[2, ::29] = np.float32(1e-40)
    big = torch.full((d, ld), 7.0, dtype=torch.float32)
    big[:, :n] = torch.from_numpy(x)
    kw = dict(leaf_size=24, num_subsets=8, split_rule=rule, key_rule=key)
    o = oracle_tree(x, **kw)
    for pts_out in (True, False):
        t = kdtree.build(big.cuda()[:, :n], points_out=pts_out, **kw)
        torch.cuda.synchronize()
        g = t.to_numpy()
        if pts_out:
            assert_same_tree(g, o, x)
        else:
            assert_same_tree(g, o)


def test_workspace_too_small_rejected_before_any_work():
    import ctypes

    import torch

    from paper_2201_08288_amd import kdtree
    print("case small workspace", flush=True)
    x = torch.from_numpy(synth.uniform24(10000, 3, seed=2)).cuda()
    prm = kdtree.make_params(leaf_size=16)
    cap, ws = kdtree.tree_bounds(10000, 3, prm)
    prm.node_capacity = cap
    tree = kdtree.KDTree(10000, 3, cap, x.device)
    tree.hdr.fill_(7)
    small = torch.empty(ws - 1, dtype=torch.uint8, device="cuda")
    st = kdtree.lib().kd_build(x.data_ptr(), 10000, 3, 10000, ctypes.byref(prm),
                               ctypes.byref(tree.struct), small.data_ptr(), small.numel(), None)
    assert st == kdtree.KD_ENOMEM
    torch.cuda.synchronize()
    assert (tree.hdr.cpu() == 7).all()  # nothing was enqueued
    # a null argument is rejected the same way
    assert kdtree.lib().kd_build(None, 10000, 3, 10000, ctypes.byref(prm), ctypes.byref(tree.struct),
                                 small.data_ptr(), small.numel(), None) == kdtree.KD_EINVAL
