"""Thin Python binding of libkdtree.so (argument marshalling only).

Every step of the build runs in the HIP library; PyTorch only provides device
memory and the current stream.  The library must be built (``_build.build()``)
before use; loading fails loudly when it is missing and cannot be built.
"""
import ctypes
import os

import numpy as np
import torch

from . import _build

KEY_CYCLIC, KEY_MAXVAR = 0, 1
SPLIT_EXACT, SPLIT_FOURIER, SPLIT_SUBSET = 0, 1, 2
KD_OK, KD_EINVAL, KD_ENOMEM, KD_ENAN, KD_ECAPACITY, KD_EDEVICE, KD_ECANCELLED = range(7)
FLAG_LEVEL_BY_LEVEL = 1
NO_LEAF = 0xFFFFFFFF

_u32, _u64, _vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [("leaf_size", _u32), ("max_depth", _u32), ("num_subsets", _u32),
                ("key_rule", _u32), ("split_rule", _u32), ("fourier_J", _u32),
                ("subset_pool", _vp), ("pool_entries", _u32), ("flags", _u32),
                ("seed", _u64), ("node_capacity", _u64)]


class TreeStruct(ctypes.Structure):
    _fields_ = [("perm", _vp), ("node_begin", _vp), ("node_end", _vp), ("node_child", _vp),
                ("node_dim", _vp), ("node_split", _vp), ("node_split_f", _vp),
                ("node_leaf", _vp), ("leaf_node", _vp), ("leaf_offsets", _vp), ("hdr", _vp),
                ("points_out", _vp), ("node_capacity", _u64), ("n", _u64), ("d", _u32),
                ("reserved", _u32)]


PROF_KINDS = ("ingest", "select", "pick", "count", "big_scatter", "small", "emit", "other")


class KernelStat(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", _u64), ("points", _u64), ("bytes", _u64)]


class Profile(ctypes.Structure):
    _fields_ = [("k", KernelStat * len(PROF_KINDS)), ("levels", _u32), ("reserved", _u32)]

    def to_dict(self):
        out = {"levels": self.levels}
        for i, name in enumerate(PROF_KINDS):
            k = self.k[i]
            out[name] = {"ms": k.ms, "launches": k.launches, "points": k.points, "bytes": k.bytes}
        return out


class Tuning(ctypes.Structure):
    _fields_ = [("hist_blocks", _u32), ("scatter_blocks", _u32), ("small_blocks", _u32),
                ("digit_bits", _u32)]

    def to_dict(self):
        return {"hist_blocks": self.hist_blocks, "scatter_blocks": self.scatter_blocks,
                "small_blocks": self.small_blocks, "digit_bits": self.digit_bits}


class BatchItem(ctypes.Structure):
    _fields_ = [("pts", _vp), ("n", _u64), ("d", _u32), ("reserved", _u32), ("ld", _u64),
                ("out", TreeStruct)]


_lib = None


def lib():
    """Load libkdtree.so, building it first when it is missing or was built
    from other sources than the ones beside it."""
    global _lib
    if _lib is None:
        if _build.stale():
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        st = ctypes.c_int32
        L.kd_tree_bounds.restype = st
        L.kd_tree_bounds.argtypes = [_u64, _u32, ctypes.POINTER(Params), ctypes.POINTER(_u64),
                                     ctypes.POINTER(_u64)]
        L.kd_build.restype = st
        L.kd_build.argtypes = [_vp, _u64, _u32, _u64, ctypes.POINTER(Params),
                               ctypes.POINTER(TreeStruct), _vp, _u64, _vp]
        L.kd_build_noalloc.restype = st
        L.kd_build_noalloc.argtypes = [_vp, _u64, _u32, _u64, ctypes.POINTER(Params),
                                       ctypes.POINTER(TreeStruct), _vp]
        L.kd_build_profiled.restype = st
        L.kd_build_profiled.argtypes = [_vp, _u64, _u32, _u64, ctypes.POINTER(Params),
                                        ctypes.POINTER(TreeStruct), _vp, _u64, _vp,
                                        ctypes.POINTER(Profile)]
        L.kd_batch_bounds.restype = st
        L.kd_batch_bounds.argtypes = [_u32, ctypes.POINTER(BatchItem), ctypes.POINTER(Params),
                                      ctypes.POINTER(_u64)]
        L.kd_build_batched.restype = st
        L.kd_build_batched.argtypes = [_u32, ctypes.POINTER(BatchItem), ctypes.POINTER(Params),
                                       _vp, _u64, _vp]
        L.kd_query_leaf.restype = st
        L.kd_query_leaf.argtypes = [ctypes.POINTER(TreeStruct), _vp, _u64, _u32, _u64, _vp, _vp]
        L.kd_query_knn.restype = st
        L.kd_query_knn.argtypes = [ctypes.POINTER(TreeStruct), _u64, _vp, _u64, _u32, _u64, _u32,
                                   _vp, _vp, _vp]
        L.kd_query_box.restype = st
        L.kd_query_box.argtypes = [ctypes.POINTER(TreeStruct), _u64, _vp, _vp, _u64, _u32, _u64,
                                   _vp, _vp, _vp, _vp]
        L.kd_global_moments.restype = st
        L.kd_global_moments.argtypes = [_vp, _u64, _u32, _u64, _u32, _vp, _vp]
        L.kd_global_solve.restype = st
        L.kd_global_solve.argtypes = [_vp, _u32, _u32, _u32, _vp, _vp]
        L.kd_global_counts.restype = st
        L.kd_global_counts.argtypes = [_vp, _u64, _u32, _u64, _vp, _u32, _vp, _vp]
        L.kd_set_tuning.restype = st
        L.kd_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.kd_get_tuning.restype = st
        L.kd_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.kd_autotune.restype = st
        L.kd_autotune.argtypes = [_vp, _u64, _u32, _u64, ctypes.POINTER(Params),
                                  ctypes.POINTER(TreeStruct), _vp, _u64, _vp,
                                  ctypes.POINTER(Tuning)]
        L.kd_status_string.restype = ctypes.c_char_p
        L.kd_status_string.argtypes = [st]
        L.kd_version.restype = ctypes.c_int
        _lib = L
    return _lib


class KDError(RuntimeError):
    def __init__(self, status, what):
        msg = lib().kd_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})")
        self.status = status


def _check(status, what):
    if status != KD_OK:
        raise KDError(status, what)


def make_params(leaf_size=32, max_depth=0, num_subsets=1, key_rule=KEY_CYCLIC,
                split_rule=SPLIT_EXACT, fourier_J=15, subset_pool=None, seed=0,
                node_capacity=0, flags=0):
    p = Params()
    p.flags = flags
    p.leaf_size = leaf_size
    p.max_depth = max_depth
    p.num_subsets = num_subsets
    p.key_rule = key_rule
    p.split_rule = split_rule
    p.fourier_J = fourier_J
    if subset_pool is not None:
        assert subset_pool.is_cuda and subset_pool.dtype == torch.int32 and subset_pool.dim() == 2
        assert subset_pool.shape[1] == num_subsets and subset_pool.is_contiguous()
        p.subset_pool = subset_pool.data_ptr()
        p.pool_entries = subset_pool.shape[0]
    p.seed = seed
    p.node_capacity = node_capacity
    return p


def tree_bounds(n, d, params):
    cap, ws = _u64(), _u64()
    _check(lib().kd_tree_bounds(n, d, ctypes.byref(params), ctypes.byref(cap), ctypes.byref(ws)),
           "kd_tree_bounds")
    return cap.value, ws.value


class KDTree:
    """Device arrays of one built tree (torch tensors, int32 storage of uint32)."""

    FIELDS = ("perm", "node_begin", "node_end", "node_child", "node_dim", "node_split",
              "node_split_f", "node_leaf", "leaf_node", "leaf_offsets")

    def __init__(self, n, d, cap, device, points_out=True):
        z = lambda m, dt=torch.int32: torch.empty(m, dtype=dt, device=device)
        self.n, self.d, self.cap = n, d, cap
        self.perm = z(n)
        self.node_begin, self.node_end = z(cap), z(cap)
        self.node_child, self.node_dim, self.node_split = z(cap), z(cap), z(cap)
        self.node_split_f = z(cap, torch.float32)
        self.node_leaf, self.leaf_node = z(cap), z(cap)
        self.leaf_offsets = z(cap + 1)
        self.hdr = torch.zeros(8, dtype=torch.int32, device=device)
        self.points_out = z((d, n), torch.float32) if points_out else None
        self.struct = TreeStruct()
        for f in self.FIELDS:
            setattr(self.struct, f, getattr(self, f).data_ptr())
        self.struct.hdr = self.hdr.data_ptr()
        self.struct.points_out = self.points_out.data_ptr() if points_out else None
        self.struct.node_capacity = cap
        self.struct.n = n
        self.struct.d = d

    def header(self):
        h = self.hdr.cpu().numpy()
        return {"num_nodes": int(np.uint32(h[0])), "num_leaves": int(np.uint32(h[1])),
                "depth": int(np.uint32(h[2])), "status": int(h[3]),
                "point_levels": int(h[4:6].view(np.uint64)[0]),
                "unsplittable": int(np.uint32(h[6])), "oversize": int(np.uint32(h[7]))}

    def to_numpy(self):
        """Host copy in the oracle's dict layout (arrays trimmed to the tree)."""
        h = self.header()
        nn, nl = h["num_nodes"], h["num_leaves"]
        u = lambda t, m: t[:m].cpu().numpy().view(np.uint32)
        out = dict(h)
        out["perm"] = u(self.perm, self.n)
        for f in ("node_begin", "node_end", "node_dim", "node_split", "node_leaf"):
            out[f] = u(getattr(self, f), nn)
        out["node_child"] = self.node_child[:nn].cpu().numpy()
        out["node_split_f"] = self.node_split_f[:nn].cpu().numpy()
        out["leaf_node"] = u(self.leaf_node, nl)
        out["leaf_offsets"] = u(self.leaf_offsets, nl + 1)
        if self.points_out is not None:
            out["points_out"] = self.points_out.cpu().numpy()
        return out


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def build(points, leaf_size=32, max_depth=0, num_subsets=1, key_rule=KEY_CYCLIC,
          split_rule=SPLIT_EXACT, fourier_J=15, subset_pool=None, seed=0, node_capacity=0,
          points_out=True, workspace=None, stream=None, tree=None, profile=None, flags=0):
    """kd_build on a (d, ld)-strided float32 CUDA tensor of shape (d, n).

    tree: reuse the output arrays of an earlier KDTree of the same shape.
    profile: a Profile() to fill with per-kernel HIP-event timings.
    """
    assert points.is_cuda and points.dtype == torch.float32 and points.dim() == 2
    assert points.stride(1) == 1
    d, n = points.shape
    ld = points.stride(0) if d > 1 else n
    prm = make_params(leaf_size, max_depth, num_subsets, key_rule, split_rule, fourier_J,
                      subset_pool, seed, node_capacity, flags)
    cap, _ = tree_bounds(n, d, prm)
    if tree is None or tree.cap < cap or tree.n != n or tree.d != d:
        tree = KDTree(n, d, cap, points.device, points_out)
    # the build may use all of a reused tree's node arrays: size the workspace for them
    prm.node_capacity = tree.cap
    _, ws = tree_bounds(n, d, prm)
    if workspace is None or workspace.numel() < ws:
        workspace = torch.empty(ws, dtype=torch.uint8, device=points.device)
    if profile is None:
        st = lib().kd_build(points.data_ptr(), n, d, ld, ctypes.byref(prm),
                            ctypes.byref(tree.struct), workspace.data_ptr(), workspace.numel(),
                            _stream_ptr(stream))
    else:
        st = lib().kd_build_profiled(points.data_ptr(), n, d, ld, ctypes.byref(prm),
                                     ctypes.byref(tree.struct), workspace.data_ptr(),
                                     workspace.numel(), _stream_ptr(stream),
                                     ctypes.byref(profile))
    _check(st, "kd_build")
    tree.params = prm
    tree.workspace = workspace
    return tree


NOALLOC_SCRATCH_BYTES = 64 << 20


def build_noalloc(points, tree, leaf_size=32, max_depth=0, num_subsets=1, key_rule=KEY_CYCLIC,
                  split_rule=SPLIT_EXACT, fourier_J=15, subset_pool=None, seed=0, stream=None,
                  flags=0):
    """kd_build_noalloc into an existing KDTree (the library's fixed per-device
    workspace; nothing is allocated)."""
    assert points.is_cuda and points.dtype == torch.float32 and points.dim() == 2
    assert points.stride(1) == 1
    d, n = points.shape
    assert tree.n == n and tree.d == d
    ld = points.stride(0) if d > 1 else n
    prm = make_params(leaf_size, max_depth, num_subsets, key_rule, split_rule, fourier_J,
                      subset_pool, seed, tree.cap, flags)
    _check(lib().kd_build_noalloc(points.data_ptr(), n, d, ld, ctypes.byref(prm),
                                  ctypes.byref(tree.struct), _stream_ptr(stream)),
           "kd_build_noalloc")
    tree.params = prm
    return tree


def build_batched(points_list, leaf_size=32, max_depth=0, num_subsets=1, key_rule=KEY_CYCLIC,
                  split_rule=SPLIT_EXACT, fourier_J=15, subset_pool=None, seed=0,
                  node_capacity=0, points_out=True, workspace=None, stream=None, flags=0):
    """kd_build_batched over a list of (d_t, n_t) float32 CUDA tensors
    (node_capacity: node-array entries of every tree, 0 = the default)."""
    prm = make_params(leaf_size, max_depth, num_subsets, key_rule, split_rule, fourier_J,
                      subset_pool, seed, node_capacity, flags)
    T = len(points_list)
    items = (BatchItem * T)()
    trees = []
    for t, pts in enumerate(points_list):
        assert pts.is_cuda and pts.dtype == torch.float32 and pts.stride(1) == 1
        d, n = pts.shape
        cap, _ = tree_bounds(n, d, prm)
        tr = KDTree(n, d, cap, pts.device, points_out)
        trees.append(tr)
        items[t].pts = pts.data_ptr()
        items[t].n = n
        items[t].d = d
        items[t].ld = pts.stride(0) if d > 1 else n
        items[t].out = tr.struct
    ws = _u64()
    _check(lib().kd_batch_bounds(T, items, ctypes.byref(prm), ctypes.byref(ws)), "kd_batch_bounds")
    if workspace is None or workspace.numel() < ws.value:
        workspace = torch.empty(ws.value, dtype=torch.uint8, device=points_list[0].device)
    _check(lib().kd_build_batched(T, items, ctypes.byref(prm), workspace.data_ptr(),
                                  workspace.numel(), _stream_ptr(stream)), "kd_build_batched")
    for tr in trees:
        tr.params = prm
    return trees


def query_leaf(tree, queries, stream=None):
    """kd_query_leaf: leaf index (int32 storage of uint32) of each query column."""
    assert queries.is_cuda and queries.dtype == torch.float32 and queries.stride(1) == 1
    d, nq = queries.shape
    assert d == tree.d, f"queries have {d} coordinates, the tree {tree.d}"
    out = torch.empty(nq, dtype=torch.int32, device=queries.device)
    ldq = queries.stride(0) if d > 1 else nq
    _check(lib().kd_query_leaf(ctypes.byref(tree.struct), queries.data_ptr(), nq, d, ldq,
                               out.data_ptr(), _stream_ptr(stream)), "kd_query_leaf")
    return out


def _query_cols(x):
    assert x.is_cuda and x.dtype == torch.float32 and x.stride(1) == 1
    d, m = x.shape
    return d, m, (x.stride(0) if d > 1 else m)


def query_knn(tree, queries, k, stream=None):
    """kd_query_knn: (indices int32 [nq, k] holding uint32, squared distances
    float64 [nq, k]) of the k nearest tree points of each query column.  The
    tree must have been built with points_out."""
    d, nq, ldq = _query_cols(queries)
    assert d == tree.d, f"queries have {d} coordinates, the tree {tree.d}"
    idx = torch.empty((nq, k), dtype=torch.int32, device=queries.device)
    dist = torch.empty((nq, k), dtype=torch.float64, device=queries.device)
    _check(lib().kd_query_knn(ctypes.byref(tree.struct), tree.n, queries.data_ptr(), nq, d, ldq,
                              k, idx.data_ptr(), dist.data_ptr(), _stream_ptr(stream)),
           "kd_query_knn")
    return idx, dist


def query_box(tree, lo, hi, ids=False, stream=None):
    """kd_query_box: points of the tree inside each box [lo, hi] (columns of
    two [d, nb] tensors).  Returns counts (int32 [nb]); with ids=True also
    (offsets int64 [nb], original indices int32 [total]) from a second call."""
    d, nb, ldb = _query_cols(lo)
    assert d == tree.d, f"boxes have {d} coordinates, the tree {tree.d}"
    assert hi.shape == lo.shape and hi.stride() == lo.stride()
    cnt = torch.empty(nb, dtype=torch.int32, device=lo.device)
    L = lib()
    _check(L.kd_query_box(ctypes.byref(tree.struct), tree.n, lo.data_ptr(), hi.data_ptr(), nb, d,
                          ldb, cnt.data_ptr(), None, None, _stream_ptr(stream)), "kd_query_box")
    if not ids:
        return cnt
    c64 = cnt.to(torch.int64)
    off = torch.cumsum(c64, 0) - c64
    total = int(c64.sum().item()) if nb else 0
    out = torch.empty(max(total, 1), dtype=torch.int32, device=lo.device)
    cnt2 = torch.empty_like(cnt)
    _check(L.kd_query_box(ctypes.byref(tree.struct), tree.n, lo.data_ptr(), hi.data_ptr(), nb, d,
                          ldb, cnt2.data_ptr(), off.data_ptr(), out.data_ptr(), _stream_ptr(stream)),
           "kd_query_box")
    return cnt, off, out[:total]


def global_moments(points, J=15, moments=None, stream=None):
    """kd_global_moments over the columns of a (p, ld)-strided float32 CUDA
    tensor of points in (0,1)^p; adds to `moments` (int64 [(2J+1)^p], a new
    zeroed tensor if None) and returns it."""
    d, n, ld = _query_cols(points)
    if moments is None:
        moments = torch.zeros((2 * J + 1) ** d, dtype=torch.int64, device=points.device)
    _check(lib().kd_global_moments(points.data_ptr(), n, d, ld, J, moments.data_ptr(),
                                   _stream_ptr(stream)), "kd_global_moments")
    return moments


def global_solve(moments, p, J=15, depth=6, stream=None):
    """kd_global_solve: the 2^depth - 1 medians (float64, heap order)."""
    med = torch.empty((1 << depth) - 1, dtype=torch.float64, device=moments.device)
    _check(lib().kd_global_solve(moments.data_ptr(), p, J, depth, med.data_ptr(),
                                 _stream_ptr(stream)), "kd_global_solve")
    return med


def global_counts(points, medians, depth, stream=None):
    """kd_global_counts: points per leaf cell (int64 [2^depth])."""
    d, n, ld = _query_cols(points)
    cnt = torch.empty(1 << depth, dtype=torch.int64, device=points.device)
    _check(lib().kd_global_counts(points.data_ptr(), n, d, ld, medians.data_ptr(), depth,
                                  cnt.data_ptr(), _stream_ptr(stream)), "kd_global_counts")
    return cnt


def set_tuning(hist_blocks=0, scatter_blocks=0, small_blocks=0, digit_bits=0):
    """kd_set_tuning: process-wide launch shapes and digit width (0 = default)."""
    t = Tuning(hist_blocks, scatter_blocks, small_blocks, digit_bits)
    _check(lib().kd_set_tuning(ctypes.byref(t)), "kd_set_tuning")


def get_tuning():
    t = Tuning()
    _check(lib().kd_get_tuning(ctypes.byref(t)), "kd_get_tuning")
    return t.to_dict()


def autotune(points, leaf_size=32, max_depth=0, num_subsets=1, key_rule=KEY_CYCLIC,
             split_rule=SPLIT_EXACT, fourier_J=15, subset_pool=None, seed=0, stream=None,
             flags=0):
    """kd_autotune on this input; returns the chosen launch shapes (now in use)."""
    assert points.is_cuda and points.dtype == torch.float32 and points.stride(1) == 1
    d, n = points.shape
    ld = points.stride(0) if d > 1 else n
    prm = make_params(leaf_size, max_depth, num_subsets, key_rule, split_rule, fourier_J,
                      subset_pool, seed, 0, flags)
    cap, ws = tree_bounds(n, d, prm)
    prm.node_capacity = cap
    workspace = torch.empty(ws, dtype=torch.uint8, device=points.device)
    tree = KDTree(n, d, cap, points.device, False)
    best = Tuning()
    _check(lib().kd_autotune(points.data_ptr(), n, d, ld, ctypes.byref(prm),
                             ctypes.byref(tree.struct), workspace.data_ptr(), workspace.numel(),
                             _stream_ptr(stream), ctypes.byref(best)), "kd_autotune")
    return best.to_dict()


def version():
    return lib().kd_version()
