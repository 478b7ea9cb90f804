"""Helpers for the GPU parity tests: build through the C ABI, compare with the
oracle element by element."""
import numpy as np

import oracle

TREE_KEYS = ("perm", "node_begin", "node_end", "node_child", "node_dim", "node_split",
             "node_leaf", "leaf_node", "leaf_offsets")
HDR_KEYS = ("status", "num_nodes", "num_leaves", "depth", "point_levels", "unsplittable",
            "oversize")

RULES = {"exact": 0, "fourier": 1, "subset": 2}
KEYS = {"cyclic": 0, "maxvar": 1}


def gpu_tree(x, **kw):
    import torch

    from paper_2201_08288_amd import kdtree
    pool = kw.pop("pool", None)
    if pool is not None:
        kw["subset_pool"] = torch.from_numpy(np.ascontiguousarray(pool).view(np.int32)).cuda()
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    t = kdtree.build(xt, **kw)
    torch.cuda.synchronize()
    return t, t.to_numpy()


def oracle_tree(x, **kw):
    kw = dict(kw)
    pool = kw.pop("pool", None)
    kw.pop("points_out", None)
    return oracle.build_tree(x, pool=pool, **kw)


def assert_same_tree(g, o, x=None):
    for k in HDR_KEYS:
        assert g[k] == o[k], (k, g[k], o[k])
    for k in TREE_KEYS:
        a, b = np.asarray(g[k]), np.asarray(o[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        if not np.array_equal(a.astype(np.int64), b.astype(np.int64)):
            bad = np.nonzero(a.astype(np.int64) != b.astype(np.int64))[0]
            raise AssertionError(f"{k}: {bad.size} mismatches, first at {bad[:5]}: "
                                 f"gpu {a[bad[:5]]} oracle {b[bad[:5]]}")
    if x is not None and "points_out" in g:
        assert np.array_equal(g["points_out"].view(np.uint32),
                              np.ascontiguousarray(x)[:, g["perm"]].view(np.uint32))
    # the decoded split matches the key
    internal = g["node_child"] >= 0
    ks = g["node_split"][internal]
    bits = np.where(ks & 0x80000000, ks & 0x7FFFFFFF, ~ks).astype(np.uint32)
    assert np.array_equal(g["node_split_f"][internal].view(np.uint32), bits)
