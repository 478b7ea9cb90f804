"""Structural invariants every built tree must satisfy, whatever the split rule.

Used on oracle trees (CPU) and on GPU trees at sizes where the oracle cannot
rebuild the whole tree.  Inputs are numpy arrays in the tree dict layout.
"""
import numpy as np


def keys_of(points):
    """Order-preserving uint32 keys (-0 folded onto +0), vectorised."""
    b = np.ascontiguousarray(points, dtype=np.float32).view(np.uint32).copy()
    b[b == 0x80000000] = 0
    neg = (b & 0x80000000) != 0
    out = np.where(neg, ~b, b | np.uint32(0x80000000)).astype(np.uint32)
    return out


def check_tree(points, tree, leaf_size, max_depth=64, check_stable=True):
    d, n = points.shape
    perm = np.asarray(tree["perm"], dtype=np.int64)
    nb = np.asarray(tree["node_begin"], dtype=np.int64)
    ne = np.asarray(tree["node_end"], dtype=np.int64)
    ch = np.asarray(tree["node_child"], dtype=np.int64)
    dim = np.asarray(tree["node_dim"], dtype=np.int64)
    spl = np.asarray(tree["node_split"], dtype=np.uint32)
    nl = np.asarray(tree["node_leaf"], dtype=np.int64)
    lnode = np.asarray(tree["leaf_node"], dtype=np.int64)
    loff = np.asarray(tree["leaf_offsets"], dtype=np.int64)
    N = nb.size
    assert N == tree["num_nodes"] and lnode.size == tree["num_leaves"]
    # (i) perm is a permutation
    assert perm.size == n and np.array_equal(np.sort(perm), np.arange(n))
    assert nb[0] == 0 and ne[0] == n
    # children: consecutive ids, ranges tile the parent
    internal = np.nonzero(ch >= 0)[0]
    lc = ch[internal]
    assert (lc >= 1).all() and (lc + 1 < N).all()
    assert np.array_equal(nb[lc], nb[internal]) and np.array_equal(ne[lc + 1], ne[internal])
    assert np.array_equal(ne[lc], nb[lc + 1])
    assert (ne[lc] > nb[lc]).all() and (ne[lc + 1] > nb[lc + 1]).all()
    # every non-root node has exactly one parent; breadth-first: children after parent
    assert np.array_equal(np.sort(np.concatenate([lc, lc + 1])), np.arange(1, N))
    assert (lc > internal).all()
    # leaves tile [0, n) in position order
    leaves = np.nonzero(ch < 0)[0]
    assert leaves.size == lnode.size
    assert np.array_equal(np.sort(leaves), np.sort(lnode))
    assert np.array_equal(loff[:-1], nb[lnode]) and loff[-1] == n
    assert np.array_equal(loff[1:], ne[lnode])
    assert np.array_equal(nl[lnode], np.arange(lnode.size))
    assert (nl[internal] == 0xFFFFFFFF).all()
    # (ii) left <= split < right on the node's key, for every internal node
    keys = keys_of(points)
    kp = keys[:, perm]
    for c in np.unique(dim[internal]):
        nodes = internal[dim[internal] == c]
        row = kp[c]
        l_end = ne[ch[nodes]]
        for k, node in enumerate(nodes):
            left = row[nb[node]:l_end[k]]
            right = row[l_end[k]:ne[node]]
            assert left.max() <= spl[node] < right.min(), node
    # leaf sizes: > leaf_size only when depth cap hit or all keys equal
    sizes = ne[lnode] - nb[lnode]
    assert (sizes >= 1).all()
    # stability: original order kept inside every leaf
    if check_stable:
        for k in range(lnode.size):
            seg = perm[loff[k]:loff[k + 1]]
            assert (np.diff(seg) > 0).all()
    return True


def depth_of_nodes(tree):
    ch = np.asarray(tree["node_child"], dtype=np.int64)
    depth = np.zeros(ch.size, dtype=np.int64)
    for k in range(ch.size):
        if ch[k] >= 0:
            depth[ch[k]] = depth[k] + 1
            depth[ch[k] + 1] = depth[k] + 1
    return depth


def descend(tree, q):
    """Leaf index of each query column of q (d, nq) by descent u <= split -> left."""
    ch = np.asarray(tree["node_child"], dtype=np.int64)
    dim = np.asarray(tree["node_dim"], dtype=np.int64)
    spl = np.asarray(tree["node_split"], dtype=np.uint32)
    nl = np.asarray(tree["node_leaf"], dtype=np.int64)
    keys = keys_of(q)
    nq = q.shape[1]
    node = np.zeros(nq, dtype=np.int64)
    active = ch[node] >= 0
    while active.any():
        idx = np.nonzero(active)[0]
        nd = node[idx]
        go_right = keys[dim[nd], idx] > spl[nd]
        node[idx] = ch[nd] + go_right
        active = ch[node] >= 0
    return nl[node]
