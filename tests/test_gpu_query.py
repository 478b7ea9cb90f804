"""GPU parity of the tree queries (kd_query_knn, kd_query_box) against the
brute-force oracles: identical neighbour lists and distances bit for bit,
identical box contents, ids in tree position order."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2201_08288_amd import synth

pytestmark = pytest.mark.gpu

CASES = [  # (n, d, leaf, generator)
    (1, 1, 8, "uniform"), (7, 2, 1, "uniform"), (1000, 3, 8, "uniform"),
    (20000, 3, 32, "gmm"), (5000, 8, 16, "ties"), (30000, 16, 64, "gmm"),
    # the widest box bound (one coordinate per lane), and the plane bound beyond it
    (4000, 64, 16, "ties"), (3000, 65, 16, "gmm"), (2000, 200, 8, "gmm"),
]


def points(n, d, gen, seed):
    if gen == "uniform":
        return synth.uniform24(n, d, seed=seed)
    if gen == "gmm":
        return synth.gmm(n, d, seed=seed)
    rng = np.random.default_rng(seed)
    return rng.integers(0, 6, size=(d, n)).astype(np.float32)


def queries_for(x, m, seed):
    """Data points (distance-0 hits and ties), jittered points and far points."""
    rng = np.random.default_rng(seed)
    d, n = x.shape
    a = x[:, rng.integers(0, n, size=m)]
    b = x[:, rng.integers(0, n, size=m)] + rng.standard_normal((d, m)).astype(np.float32) * 0.05
    c = rng.standard_normal((d, m)).astype(np.float32) * 50
    return np.ascontiguousarray(np.concatenate([a, b, c], axis=1))


def built(x, leaf, **kw):
    import torch

    from paper_2201_08288_amd import kdtree
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    t = kdtree.build(xt, leaf_size=leaf, **kw)
    torch.cuda.synchronize()
    assert t.header()["status"] == 0
    return t


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("k", [1, 5, 64])
def test_knn_matches_brute_force(case, k):
    import torch

    from paper_2201_08288_amd import kdtree
    n, d, leaf, gen = CASES[case]
    print(f"case knn n={n} d={d} leaf={leaf} {gen} k={k}", flush=True)
    x = points(n, d, gen, seed=case + 40)
    t = built(x, leaf)
    q = queries_for(x, 100, seed=case)
    gi, gd = kdtree.query_knn(t, torch.from_numpy(q).cuda(), k)
    gi = gi.cpu().numpy().view(np.uint32)
    gd = gd.cpu().numpy()
    oi, od = oracle.knn(x, q, k)
    assert np.array_equal(gi, oi)
    assert np.array_equal(gd.view(np.uint64), od.view(np.uint64))


def test_knn_nan_query_and_rules():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case knn nan and fourier tree", flush=True)
    x = synth.gmm(8000, 3, seed=3)
    q = queries_for(x, 50, seed=9)
    q[1, 7] = np.nan
    for rule in (1, 2):
        t = built(x, 16, split_rule=rule, num_subsets=8)
        gi, gd = kdtree.query_knn(t, torch.from_numpy(q).cuda(), 8)
        oi, od = oracle.knn(x, q, 8)
        assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
        assert np.array_equal(np.isnan(gd.cpu().numpy()), np.isnan(od))
        ok = ~np.isnan(od)
        assert np.array_equal(gd.cpu().numpy()[ok], od[ok])


def test_knn_infinite_and_huge_query_coordinates():
    """Queries with an infinite coordinate (every distance is +inf: the list is
    the k lowest indices, so every leaf must be reached) and with coordinates
    near the float limit."""
    import torch

    from paper_2201_08288_amd import kdtree
    print("case knn infinite query coordinates", flush=True)
    x = synth.gmm(8000, 3, seed=4)
    q = queries_for(x, 20, seed=11)
    q[0, 3] = np.inf
    q[2, 4] = -np.inf
    q[:, 5] = np.float32(3.0e38)
    q[1, 6] = np.float32(-3.0e38)
    t = built(x, 16)
    for k in (1, 8, 64):
        gi, gd = kdtree.query_knn(t, torch.from_numpy(q).cuda(), k)
        oi, od = oracle.knn(x, q, k)
        assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
        assert np.array_equal(gd.cpu().numpy().view(np.uint64), od.view(np.uint64))


def boxes_for(x, m, seed):
    rng = np.random.default_rng(seed)
    d, n = x.shape
    a = x[:, rng.integers(0, n, size=m)]
    b = x[:, rng.integers(0, n, size=m)]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    lo[:, 0] = -np.inf  # everything
    hi[:, 0] = np.inf
    lo[:, 1], hi[:, 1] = hi[:, 1] + 1, lo[:, 1] - 1  # empty (lo > hi)
    lo[:, 2] = hi[:, 2] = x[:, 0]  # one point (and its duplicates)
    lo[0, 3] = np.nan
    return np.ascontiguousarray(lo), np.ascontiguousarray(hi)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_box_matches_brute_force(case):
    import torch

    from paper_2201_08288_amd import kdtree
    n, d, leaf, gen = CASES[case]
    print(f"case box n={n} d={d} leaf={leaf} {gen}", flush=True)
    x = points(n, d, gen, seed=case + 60)
    t = built(x, leaf)
    lo, hi = boxes_for(x, 64, seed=case)
    cnt, off, ids = kdtree.query_box(t, torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda(),
                                     ids=True)
    cnt = cnt.cpu().numpy()
    off = off.cpu().numpy()
    ids = ids.cpu().numpy().view(np.uint32)
    want = oracle.box_query(x, lo, hi)
    pos = np.empty(n, dtype=np.int64)
    pos[t.perm.cpu().numpy().view(np.uint32)] = np.arange(n)
    for i, w in enumerate(want):
        assert cnt[i] == w.size, (i, cnt[i], w.size)
        got = ids[off[i]:off[i] + cnt[i]]
        assert np.array_equal(np.sort(got), w)
        assert (np.diff(pos[got]) > 0).all()  # tree position order


def test_query_argument_errors():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case query errors", flush=True)
    x = synth.uniform24(1000, 2, seed=1)
    t = built(x, 8)
    q = torch.from_numpy(queries_for(x, 4, seed=1)).cuda()
    L = kdtree.lib()
    out_i = torch.empty((12, 65), dtype=torch.int32, device="cuda")
    out_d = torch.empty((12, 65), dtype=torch.float64, device="cuda")
    for k in (0, 65):
        assert L.kd_query_knn(ctypes.byref(t.struct), 1000, q.data_ptr(), 12, 2, 12, k,
                              out_i.data_ptr(), out_d.data_ptr(), None) == kdtree.KD_EINVAL
    bare = kdtree.build(torch.from_numpy(x).cuda(), leaf_size=8, points_out=False)
    assert L.kd_query_knn(ctypes.byref(bare.struct), 1000, q.data_ptr(), 12, 2, 12, 4,
                          out_i.data_ptr(), out_d.data_ptr(), None) == kdtree.KD_EINVAL
    cnt = torch.empty(12, dtype=torch.int32, device="cuda")
    assert L.kd_query_box(ctypes.byref(t.struct), 1000, q.data_ptr(), q.data_ptr(), 12, 2, 12,
                          cnt.data_ptr(), None, cnt.data_ptr(), None) == kdtree.KD_EINVAL
    torch.cuda.synchronize()
