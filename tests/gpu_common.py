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


def node_depths(child):
    """Depth of every node from the BFS child links."""
    ch = np.asarray(child, dtype=np.int64)
    dep = np.zeros(ch.size, dtype=np.int64)
    for k in range(ch.size):  # children have larger ids than their parent
        if ch[k] >= 0:
            dep[ch[k]] = dep[ch[k] + 1] = dep[k] + 1
    return dep


def level_ranks(g, leaf_size, max_depth=64):
    """Depth of every node and its rank among the cells processed at its
    depth (cells with more than leaf_size points above max_depth, ordered
    by first position) -- the rank that picks a subset-pool row."""
    nb = np.asarray(g["node_begin"], dtype=np.int64)
    size = np.asarray(g["node_end"], dtype=np.int64) - nb
    dep = node_depths(g["node_child"])
    active = (size > leaf_size) & (dep < max_depth)
    rank = np.full(nb.size, -1, dtype=np.int64)
    for dd in np.unique(dep[active]):
        ids = np.nonzero(active & (dep == dd))[0]
        order = ids[np.argsort(nb[ids], kind="stable")]
        rank[order] = np.arange(order.size)
    return dep, rank, active


def check_sampled_nodes(x, g, nodes, leaf_size, shift=0, log=None, workers=8, **kw):
    """Recompute the split of each sampled node with the oracle on that
    node's points and compare key, split and leaf status with the GPU tree.

    A cell's points at its level are in ascending original index: the root
    starts in index order and every partition is stable.  Nodes are checked
    in parallel threads (the oracle call releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    dep, rank, active = level_ranks(g, leaf_size, kw.get("max_depth", 0) or 64)
    perm = np.asarray(g["perm"])
    todo = [int(k) for k in nodes if active[int(k)]]

    def one(k):
        idx = np.sort(perm[g["node_begin"][k]:g["node_end"][k]])
        ok, dim, split, _ = oracle.cell_split(x, idx, depth=int(dep[k]), rank=int(rank[k]),
                                              shift=shift, leaf_size=leaf_size, **kw)
        internal = bool(g["node_child"][k] >= 0)
        got = (internal, int(g["node_dim"][k]), int(g["node_split"][k])) if internal else \
            (internal,)
        want = (ok, dim, split) if ok else (ok,)
        if log is not None:
            log(f"node {k} depth {dep[k]} size {idx.size}: {'ok' if got == want else 'MISMATCH'}")
        return k, got, want

    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, todo))
    bad = [r for r in res if r[1] != r[2]]
    assert not bad, f"{len(bad)} mismatching nodes, first (node, gpu, oracle): {bad[:3]}"
    return len(res)
