"""Independent pure-Python brute force of the tree build, for tiny inputs.

Written separately from the C oracle (recursive over cells instead of level by
level, Python sorting, exact rational variance, candidate enumeration for the
tie rule) so that the two can pin each other on small cases.
"""
import struct
from fractions import Fraction

import numpy as np


def f32_bits(x):
    return struct.unpack("<I", struct.pack("<f", float(x)))[0]


def order_key(x):
    """Rank-preserving integer for a float32 value: Python's own float order."""
    return float(np.float32(x)) + 0.0  # -0.0 + 0.0 == +0.0


def lower_median_value(vals):
    s = sorted(vals)
    return s[(len(s) - 1) // 2]


def choose_split(vals, m):
    """Closest-to-balanced valid split among "x <= m" and "x < m".

    Returns ("le"|"lt", left_count) or None.  Ties in balance go to "le".
    """
    n = len(vals)
    le = sum(1 for v in vals if v <= m)
    lt = sum(1 for v in vals if v < m)
    cands = []
    if 0 < le < n:
        cands.append((abs(2 * le - n), 0, "le", le))
    if 0 < lt < n:
        cands.append((abs(2 * lt - n), 1, "lt", lt))
    if not cands:
        return None
    cands.sort()
    return cands[0][2], cands[0][3]


def exact_variance_key(points, idx):
    d = points.shape[0]
    best, bestv = 0, None
    for c in range(d):
        xs = [Fraction(float(points[c, i])) for i in idx]
        mu = sum(xs) / len(xs)
        v = sum((x - mu) ** 2 for x in xs)
        if bestv is None or v > bestv:
            best, bestv = c, v
    return best


def subset_mean_of_medians(vals, S):
    n = len(vals)
    acc = 0.0
    for r in range(S):
        lo, hi = (r * n) // S, ((r + 1) * n) // S
        if hi == lo:
            continue
        med = lower_median_value(vals[lo:hi])
        acc = acc + float(hi - lo) * med
    return float(np.float32(acc / n))


def build(points, leaf_size, key="cyclic", rule="exact", S=1, max_depth=64):
    """Returns (nodes, perm) with nodes in breadth-first order.

    node = dict(begin, end, child, dim, split_value(float or None), kind)
    """
    d, n = points.shape
    perm = list(range(n))
    root = {"begin": 0, "end": n, "depth": 0, "idx": list(range(n))}
    tree = []  # (node, children) recursion results

    def rec(cell):
        idx = cell["idx"]
        nc = len(idx)
        node = {"begin": cell["begin"], "end": cell["end"], "depth": cell["depth"],
                "child": None, "dim": 0, "split": None, "kind": None, "idx": idx}
        if nc <= leaf_size or cell["depth"] >= max_depth:
            return node
        t = cell["depth"] % d if key == "cyclic" else exact_variance_key(points, idx)
        vals = [order_key(points[t, i]) for i in idx]
        if rule == "exact":
            m = lower_median_value(vals)
        elif rule == "subset":
            m = subset_mean_of_medians(vals, S)
        else:
            raise ValueError(rule)
        ch = choose_split(vals, m)
        if ch is None:
            return node
        kind, nl = ch
        if kind == "le":
            left = [i for i, v in zip(idx, vals) if v <= m]
            right = [i for i, v in zip(idx, vals) if v > m]
        else:
            left = [i for i, v in zip(idx, vals) if v < m]
            right = [i for i, v in zip(idx, vals) if v >= m]
        assert len(left) == nl
        node["dim"], node["split"], node["kind"] = t, m, kind
        b = cell["begin"]
        lc = rec({"begin": b, "end": b + nl, "depth": cell["depth"] + 1, "idx": left})
        rc = rec({"begin": b + nl, "end": cell["end"], "depth": cell["depth"] + 1, "idx": right})
        node["child"] = (lc, rc)
        return node

    top = rec(root)
    # breadth-first numbering
    order, frontier = [], [top]
    while frontier:
        order.extend(frontier)
        nxt = []
        for nd in frontier:
            if nd["child"] is not None:
                nxt.extend(nd["child"])
        frontier = nxt
    ids = {id(nd): k for k, nd in enumerate(order)}
    out = []
    for nd in order:
        out.append({"begin": nd["begin"], "end": nd["end"],
                    "child": -1 if nd["child"] is None else ids[id(nd["child"][0])],
                    "dim": nd["dim"], "split": nd["split"], "kind": nd["kind"],
                    "depth": nd["depth"]})
        if nd["child"] is None:
            perm[nd["begin"]:nd["end"]] = nd["idx"]
    return out, perm
