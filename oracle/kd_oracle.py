"""ctypes wrapper around ``kd_oracle.c``, the plain CPU reference build.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU product path.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libkd_oracle.so")

KEY_CYCLIC, KEY_MAXVAR = 0, 1
SPLIT_EXACT, SPLIT_FOURIER, SPLIT_SUBSET = 0, 1, 2
OK, EINVAL, ENOMEM, ENONFINITE, ECAPACITY = 0, 1, 2, 3, 4

_CFLAGS = ["-O2", "-march=x86-64-v2", "-std=gnu11", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared"]


def build():
    """Compile the oracle with gcc (contraction off, no fast-math, OpenMP)."""
    subprocess.check_call(["gcc", *_CFLAGS, "-o", _LIB_PATH, _SRC, "-lm"])


class Params(ctypes.Structure):
    _fields_ = [
        ("leaf_size", ctypes.c_uint32),
        ("max_depth", ctypes.c_uint32),
        ("num_subsets", ctypes.c_uint32),
        ("key_rule", ctypes.c_uint32),
        ("split_rule", ctypes.c_uint32),
        ("fourier_J", ctypes.c_uint32),
        ("pool", ctypes.c_void_p),
        ("pool_entries", ctypes.c_uint32),
        ("pad_", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("node_capacity", ctypes.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u32, u64, i32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p
        L.kdo_key_of_bits.restype = u32
        L.kdo_key_of_bits.argtypes = [u32]
        L.kdo_bits_of_key.restype = u32
        L.kdo_bits_of_key.argtypes = [u32]
        L.kdo_splitmix64.restype = u64
        L.kdo_splitmix64.argtypes = [u64]
        L.kdo_lower_median.restype = u32
        L.kdo_lower_median.argtypes = [vp, u64]
        L.kdo_tie_rule.restype = ctypes.c_int
        L.kdo_tie_rule.argtypes = [u64, u64, u64, u32, ctypes.POINTER(u32)]
        L.kdo_subset_bounds.restype = None
        L.kdo_subset_bounds.argtypes = [u64, u32, vp, u32, u64, u32, u64, vp]
        L.kdo_maxvar_shift.restype = ctypes.c_int
        L.kdo_maxvar_shift.argtypes = [vp, u64, u32, u64]
        L.kdo_maxvar_key.restype = u32
        L.kdo_maxvar_key.argtypes = [vp, u32, u64, vp, u64, ctypes.c_int]
        L.kdo_sincos_f32.restype = None
        L.kdo_sincos_f32.argtypes = [ctypes.c_float, ctypes.POINTER(ctypes.c_float),
                                     ctypes.POINTER(ctypes.c_float)]
        L.kdo_sincos_f64.restype = None
        L.kdo_sincos_f64.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
        L.kdo_fourier_exponent.restype = ctypes.c_int
        L.kdo_fourier_exponent.argtypes = [u32, u32]
        L.kdo_fourier_map.restype = None
        L.kdo_fourier_map.argtypes = [vp, u64, u32, ctypes.c_int, u32, vp, vp]
        L.kdo_fourier_F.restype = ctypes.c_double
        L.kdo_fourier_F.argtypes = [vp, vp, u32, ctypes.c_double]
        L.kdo_fourier_solve.restype = u32
        L.kdo_fourier_solve.argtypes = [vp, vp, u32, u32, u32, ctypes.c_int]
        L.kdo_cell_split.restype = ctypes.c_int
        L.kdo_cell_split.argtypes = [vp, u32, u64, ctypes.POINTER(Params), ctypes.c_int, vp, u64,
                                     u32, u64, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                     ctypes.POINTER(u32)]
        L.kdo_build.restype = ctypes.c_int
        L.kdo_build.argtypes = [vp, u64, u32, u64, ctypes.POINTER(Params)] + [vp] * 10
        L.kdo_set_threads.restype = ctypes.c_int
        L.kdo_set_threads.argtypes = [ctypes.c_int]
        L.kdo_build_batched.restype = None
        L.kdo_build_batched.argtypes = [u32, vp, vp, vp, vp, vp, vp]
        L.kdo_check_partition.restype = u64
        L.kdo_check_partition.argtypes = [vp, u32, u64, vp, u64, vp, vp, vp, vp, vp]
        L.kdo_query_leaf.restype = u32
        L.kdo_query_leaf.argtypes = [vp, vp, vp, vp, vp, u64]
        L.kdo_global_quantum.restype = ctypes.c_float
        L.kdo_global_quantum.argtypes = [u32]
        L.kdo_global_basis.restype = None
        L.kdo_global_basis.argtypes = [ctypes.c_float, u32, ctypes.c_float, vp]
        L.kdo_global_g.restype = None
        L.kdo_global_g.argtypes = [ctypes.c_double, ctypes.c_double, u32, vp]
        L.kdo_global_moments.restype = None
        L.kdo_global_moments.argtypes = [vp, u64, u32, u64, u32, vp]
        L.kdo_global_solve.restype = None
        L.kdo_global_solve.argtypes = [vp, u32, u32, u32, vp]
        L.kdo_global_counts.restype = None
        L.kdo_global_counts.argtypes = [vp, u64, u32, u64, vp, u32, vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# ---------------------------------------------------------------- primitives

def key_of_bits(b):
    return lib().kdo_key_of_bits(int(b) & 0xFFFFFFFF)


def bits_of_key(u):
    return lib().kdo_bits_of_key(int(u) & 0xFFFFFFFF)


def keys_of_floats(x):
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).ravel()
    return np.array([key_of_bits(v) for v in b], dtype=np.uint32)


def splitmix64(x):
    return lib().kdo_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF)


def lower_median(keys):
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    return lib().kdo_lower_median(_ptr(k), k.size)


def tie_rule(n, lt, le, m):
    s = ctypes.c_uint32(0)
    ok = lib().kdo_tie_rule(n, lt, le, int(m) & 0xFFFFFFFF, ctypes.byref(s))
    return (True, s.value) if ok else (False, None)


def subset_bounds(n, S, pool=None, seed=0, depth=0, rank=0):
    out = np.zeros(S + 1, dtype=np.uint64)
    pool_arr = None if pool is None else np.ascontiguousarray(pool, dtype=np.uint32)
    P = 0 if pool_arr is None else pool_arr.shape[0]
    lib().kdo_subset_bounds(n, S, _ptr(pool_arr), P, seed, depth, rank, _ptr(out))
    return out


def maxvar_shift(points):
    p = np.ascontiguousarray(points, dtype=np.float32)
    d, n = p.shape
    return lib().kdo_maxvar_shift(_ptr(p), n, d, n)


def maxvar_key(points, idx, shift):
    p = np.ascontiguousarray(points, dtype=np.float32)
    d, n = p.shape
    ix = np.ascontiguousarray(idx, dtype=np.uint32)
    return lib().kdo_maxvar_key(_ptr(p), d, n, _ptr(ix), ix.size, shift)


def sincos_f32(x):
    s, c = ctypes.c_float(), ctypes.c_float()
    lib().kdo_sincos_f32(float(x), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def sincos_f64(x):
    s, c = ctypes.c_double(), ctypes.c_double()
    lib().kdo_sincos_f64(float(x), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def fourier_exponent(lo_key, hi_key):
    return lib().kdo_fourier_exponent(lo_key, hi_key)


def fourier_map(keys, lo_key, e, J):
    k = np.ascontiguousarray(keys, dtype=np.uint32)
    Cc = np.zeros(J, dtype=np.int64)
    Cs = np.zeros(J, dtype=np.int64)
    lib().kdo_fourier_map(_ptr(k), k.size, lo_key, e, J, _ptr(Cc), _ptr(Cs))
    return Cc, Cs


def fourier_F(Cc, Cs, v):
    Cc = np.ascontiguousarray(Cc, dtype=np.int64)
    Cs = np.ascontiguousarray(Cs, dtype=np.int64)
    return lib().kdo_fourier_F(_ptr(Cc), _ptr(Cs), Cc.size, float(v))


def fourier_solve(Cc, Cs, lo_key, hi_key, e):
    Cc = np.ascontiguousarray(Cc, dtype=np.int64)
    Cs = np.ascontiguousarray(Cs, dtype=np.int64)
    return lib().kdo_fourier_solve(_ptr(Cc), _ptr(Cs), Cc.size, lo_key, hi_key, e)


def default_node_capacity(n, leaf_size):
    return 4 * ((n + leaf_size - 1) // leaf_size) + 64


def make_params(leaf_size=32, max_depth=0, num_subsets=1, key_rule=KEY_CYCLIC,
                split_rule=SPLIT_EXACT, fourier_J=15, pool=None, seed=0, node_capacity=0,
                n=None):
    p = Params()
    p.leaf_size = leaf_size
    p.max_depth = max_depth
    p.num_subsets = num_subsets
    p.key_rule = key_rule
    p.split_rule = split_rule
    p.fourier_J = fourier_J
    p.pool = None if pool is None else pool.ctypes.data
    p.pool_entries = 0 if pool is None else pool.shape[0]
    p.seed = seed
    if node_capacity == 0 and n is not None:
        node_capacity = default_node_capacity(n, leaf_size)
    p.node_capacity = node_capacity
    return p


def cell_split(points, idx, depth=0, rank=0, shift=0, **kw):
    """Key, split and candidate of one cell (idx: original indices in cell order)."""
    p = np.ascontiguousarray(points, dtype=np.float32)
    d, n = p.shape
    pool = kw.get("pool")
    if pool is not None:
        pool = np.ascontiguousarray(pool, dtype=np.uint32)
        kw["pool"] = pool
    prm = make_params(**kw)
    ix = np.ascontiguousarray(idx, dtype=np.uint32)
    dim, split, cand = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    ok = lib().kdo_cell_split(_ptr(p), d, n, ctypes.byref(prm), shift, _ptr(ix), ix.size,
                              depth, rank, ctypes.byref(dim), ctypes.byref(split),
                              ctypes.byref(cand))
    return bool(ok), dim.value, split.value, cand.value


def _tree_arrays(n, cap):
    return [np.zeros(n, dtype=np.uint32), np.zeros(cap, dtype=np.uint32),
            np.zeros(cap, dtype=np.uint32), np.zeros(cap, dtype=np.int32),
            np.zeros(cap, dtype=np.uint32), np.zeros(cap, dtype=np.uint32),
            np.zeros(cap, dtype=np.uint32), np.zeros(cap, dtype=np.uint32),
            np.zeros(cap + 1, dtype=np.uint32), np.zeros(7, dtype=np.uint64)]


def _tree_dict(st, arr):
    perm, nb, ne, nc, nd, ns, nl, ln, lo, hdr = arr
    nn, nlv = int(hdr[0]), int(hdr[1])
    return {
        "status": int(st), "num_nodes": nn, "num_leaves": nlv, "depth": int(hdr[2]),
        "point_levels": int(hdr[4]), "unsplittable": int(hdr[5]), "oversize": int(hdr[6]),
        "perm": perm, "node_begin": nb[:nn], "node_end": ne[:nn], "node_child": nc[:nn],
        "node_dim": nd[:nn], "node_split": ns[:nn], "node_leaf": nl[:nn],
        "leaf_node": ln[:nlv], "leaf_offsets": lo[:nlv + 1],
    }


def build_tree(points, leaf_size=32, max_depth=0, num_subsets=1, key_rule=KEY_CYCLIC,
               split_rule=SPLIT_EXACT, fourier_J=15, pool=None, seed=0, node_capacity=0):
    """Build one tree on the CPU.  points: float32 array of shape (d, n) (SoA).

    Returns a dict with perm, node_* arrays (trimmed to num_nodes), leaf_node,
    leaf_offsets (trimmed to num_leaves + 1) and header fields.
    """
    p = np.ascontiguousarray(points, dtype=np.float32)
    d, n = p.shape
    if pool is not None:
        pool = np.ascontiguousarray(pool, dtype=np.uint32)
    prm = make_params(leaf_size, max_depth, num_subsets, key_rule, split_rule, fourier_J,
                      pool, seed, node_capacity, n=n)
    arr = _tree_arrays(n, prm.node_capacity)
    st = lib().kdo_build(_ptr(p), n, d, n, ctypes.byref(prm), *[_ptr(a) for a in arr])
    return _tree_dict(st, arr)


def set_threads(nthreads):
    """OpenMP threads of the oracle's later calls (0: leave as is); returns
    the previous count.  Results do not depend on it."""
    return lib().kdo_set_threads(int(nthreads))


def build_trees(points_list, **kw):
    """Build independent trees (one per (d, n) float32 array) with the same
    parameters, trees shared out among OpenMP threads; each tree equals
    build_tree on it."""
    pts = [np.ascontiguousarray(x, dtype=np.float32) for x in points_list]
    T = len(pts)
    pool = kw.pop("pool", None)
    if pool is not None:
        pool = np.ascontiguousarray(pool, dtype=np.uint32)
    params = (Params * T)()
    arrs, outs = [], np.zeros(T * 10, dtype=np.uint64)
    for k, x in enumerate(pts):
        d, n = x.shape
        params[k] = make_params(pool=pool, n=n, **kw)
        arr = _tree_arrays(n, params[k].node_capacity)
        arrs.append(arr)
        outs[10 * k:10 * k + 10] = [a.ctypes.data for a in arr]
    ptr = np.array([x.ctypes.data for x in pts], dtype=np.uint64)
    ns = np.array([x.shape[1] for x in pts], dtype=np.uint64)
    ds = np.array([x.shape[0] for x in pts], dtype=np.uint32)
    st = np.zeros(T, dtype=np.int32)
    lib().kdo_build_batched(T, _ptr(ptr), _ptr(ns), _ptr(ds), ctypes.addressof(params),
                            _ptr(outs), _ptr(st))
    return [_tree_dict(int(st[k]), arrs[k]) for k in range(T)]


def query_leaf(tree, queries):
    """Leaf index of each query (queries: float32 (d, nq)); NaN -> 0xFFFFFFFF."""
    q = np.ascontiguousarray(queries, dtype=np.float32)
    d, nq = q.shape
    nc = np.ascontiguousarray(tree["node_child"], dtype=np.int32)
    nd = np.ascontiguousarray(tree["node_dim"], dtype=np.uint32)
    ns = np.ascontiguousarray(tree["node_split"], dtype=np.uint32)
    nl = np.ascontiguousarray(tree["node_leaf"], dtype=np.uint32)
    out = np.zeros(nq, dtype=np.uint32)
    L = lib()
    base = q.ctypes.data
    for i in range(nq):
        out[i] = L.kdo_query_leaf(_ptr(nc), _ptr(nd), _ptr(ns), _ptr(nl),
                                  ctypes.c_void_p(base + 4 * i), nq)
    return out


def check_partition(points, tree, permuted=False):
    """Number of points on the wrong side of their node's split (0 = valid).
    permuted=True: points are already in the tree's position order."""
    p = np.ascontiguousarray(points, dtype=np.float32)
    d, n = p.shape
    arr = {k: np.ascontiguousarray(tree[k], dtype=np.int32 if k == "node_child" else np.uint32)
           for k in ("node_begin", "node_end", "node_child", "node_dim", "node_split")}
    perm = None if permuted else np.ascontiguousarray(tree["perm"], dtype=np.uint32)
    return lib().kdo_check_partition(_ptr(p), d, n, _ptr(perm), arr["node_begin"].size,
                                     _ptr(arr["node_begin"]), _ptr(arr["node_end"]),
                                     _ptr(arr["node_child"]), _ptr(arr["node_dim"]),
                                     _ptr(arr["node_split"]))


# ---------------------------------------------------------------- queries
# The queries the cells of a tree serve (§1, §2: nearest neighbours, ranges),
# written as their plain definitions: brute force over every point, no tree.

QUERY_NONE = 0xFFFFFFFF


def knn(points, queries, k, chunk=256):
    """Exact k nearest neighbours by brute force.  points: float32 (d, n);
    queries: float32 (d, nq).  Squared Euclidean distance in fp64, summed
    over the coordinates in order ((x_c - q_c) rounded, squared and rounded,
    added and rounded: no fused operations); a NaN sum counts as +inf.
    Ascending by (distance, point index).  Returns (idx uint32 (nq, k),
    dist float64 (nq, k)); fewer than k points: (QUERY_NONE, +inf); a query
    with a NaN coordinate: (QUERY_NONE, NaN) throughout."""
    p = np.asarray(points, dtype=np.float32)
    q = np.asarray(queries, dtype=np.float32)
    d, n = p.shape
    nq = q.shape[1]
    idx = np.full((nq, k), QUERY_NONE, dtype=np.uint32)
    dist = np.full((nq, k), np.inf, dtype=np.float64)
    ids = np.arange(n, dtype=np.int64)
    m = min(k, n)
    for a in range(0, nq, chunk):
        b = min(nq, a + chunk)
        D = np.zeros((b - a, n), dtype=np.float64)
        for c in range(d):
            t = p[c].astype(np.float64)[None, :] - q[c, a:b].astype(np.float64)[:, None]
            D = D + t * t
        D[np.isnan(D)] = np.inf
        for r in range(b - a):
            if np.isnan(q[:, a + r]).any():
                idx[a + r] = QUERY_NONE
                dist[a + r] = np.nan
                continue
            order = np.lexsort((ids, D[r]))[:m]
            idx[a + r, :m] = order
            dist[a + r, :m] = D[r, order]
    return idx, dist


def box_query(points, lo, hi):
    """Original indices (ascending) of the points inside each box [lo, hi]:
    every coordinate within its bounds, inclusive, compared as floats (-0
    equals +0).  A box with a NaN bound holds nothing.  points: float32
    (d, n); lo, hi: float32 (d, nb).  Returns a list of uint32 arrays."""
    p = np.asarray(points, dtype=np.float32)
    lo = np.asarray(lo, dtype=np.float32)
    hi = np.asarray(hi, dtype=np.float32)
    out = []
    for i in range(lo.shape[1]):
        if np.isnan(lo[:, i]).any() or np.isnan(hi[:, i]).any():
            out.append(np.zeros(0, dtype=np.uint32))
            continue
        inside = np.all((p >= lo[:, i:i + 1]) & (p <= hi[:, i:i + 1]), axis=0)
        out.append(np.nonzero(inside)[0].astype(np.uint32))
    return out


# ---------------------------------------------------------------- global method
# The paper's single-pass construction (§3.2, Eq. (1)-(2); App. C, K = 1).


def global_quantum(p):
    """Quantum Q_p of the basis values for p coordinates."""
    return float(lib().kdo_global_quantum(p))


def global_basis(u, J, p=3):
    """Quantised basis rint(c_j(u) * Q_p), j = 0..2J, of one value in (0,1)."""
    q = np.zeros(2 * J + 1, dtype=np.float32)
    lib().kdo_global_basis(ctypes.c_float(u), J, ctypes.c_float(global_quantum(p)), _ptr(q))
    return q


def global_g(a, b, J):
    """g_0..g_{2J}(a, b) of Lemma 3.1 (fp64)."""
    g = np.zeros(2 * J + 1, dtype=np.float64)
    lib().kdo_global_g(ctypes.c_double(a), ctypes.c_double(b), J, _ptr(g))
    return g


def global_moments(points, J=15):
    """The statistics C_j, j in {0..2J}^p (int64, first coordinate slowest)
    of points in (0,1)^p (float32 (p, n))."""
    p = np.ascontiguousarray(points, dtype=np.float32)
    d, n = p.shape
    C = np.zeros((2 * J + 1) ** d, dtype=np.int64)
    lib().kdo_global_moments(_ptr(p), n, d, n, J, _ptr(C))
    return C


def global_solve(C, p, J=15, depth=6):
    """The 2^depth - 1 medians of Eq. (2), heap order (node i: children 2i+1
    on the low side, 2i+2), cycling through the coordinates by level."""
    C = np.ascontiguousarray(C, dtype=np.int64)
    med = np.zeros((1 << depth) - 1, dtype=np.float64)
    lib().kdo_global_solve(_ptr(C), p, J, depth, _ptr(med))
    return med


def global_counts(points, med, depth):
    """Points of each leaf cell (u_t <= m goes to the low side)."""
    p = np.ascontiguousarray(points, dtype=np.float32)
    d, n = p.shape
    cnt = np.zeros(1 << depth, dtype=np.uint64)
    lib().kdo_global_counts(_ptr(p), n, d, n, _ptr(np.ascontiguousarray(med, dtype=np.float64)),
                            depth, _ptr(cnt))
    return cnt


def global_build(points, J=15, depth=6):
    """Moments, medians and leaf counts of the global construction."""
    C = global_moments(points, J)
    med = global_solve(C, np.asarray(points).shape[0], J, depth)
    return {"moments": C, "medians": med, "counts": global_counts(points, med, depth)}
