"""CPU pins of the query oracles (brute-force nearest neighbours and box
search): hand-worked cases, and agreement with SciPy's own k-d tree and with
a sorting-based count."""
import numpy as np
import pytest

import oracle

NONE = oracle.QUERY_NONE


def test_knn_hand_worked_1d():
    # distances from 2 to {0, 1, 3, 3, 10}: 4, 1, 1, 1, 64 (ties by index)
    p = np.array([[0, 1, 3, 3, 10]], dtype=np.float32)
    q = np.array([[2]], dtype=np.float32)
    idx, dist = oracle.knn(p, q, 3)
    assert idx.tolist() == [[1, 2, 3]] and dist.tolist() == [[1.0, 1.0, 1.0]]
    idx, dist = oracle.knn(p, q, 7)
    assert idx.tolist() == [[1, 2, 3, 0, 4, NONE, NONE]]
    assert dist[0, :5].tolist() == [1.0, 1.0, 1.0, 4.0, 64.0] and np.isinf(dist[0, 5:]).all()


def test_knn_hand_worked_2d_and_nan_query():
    p = np.array([[0, 3, 1, -1], [0, 4, 1, 0]], dtype=np.float32)
    q = np.array([[0, np.nan], [0, 0]], dtype=np.float32)
    idx, dist = oracle.knn(p, q, 4)
    assert idx[0].tolist() == [0, 3, 2, 1] and dist[0].tolist() == [0.0, 1.0, 2.0, 25.0]
    assert (idx[1] == NONE).all() and np.isnan(dist[1]).all()


def test_knn_agrees_with_scipy_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(5)
    p = rng.standard_normal((3, 3000)).astype(np.float32)
    q = rng.standard_normal((3, 200)).astype(np.float32)
    idx, dist = oracle.knn(p, q, 10)
    sd, si = cKDTree(p.T.astype(np.float64)).query(q.T.astype(np.float64), k=10)
    assert np.array_equal(idx.astype(np.int64), si)  # continuous data: no distance ties
    assert np.allclose(dist, sd ** 2, rtol=1e-12, atol=0)


def test_knn_full_list_is_a_sorted_permutation():
    rng = np.random.default_rng(6)
    p = rng.integers(0, 4, size=(2, 50)).astype(np.float32)  # many equal distances
    q = rng.integers(0, 4, size=(2, 5)).astype(np.float32)
    idx, dist = oracle.knn(p, q, 50)
    for r in range(5):
        assert sorted(idx[r].tolist()) == list(range(50))
        pairs = list(zip(dist[r].tolist(), idx[r].tolist()))
        assert pairs == sorted(pairs)


def test_box_hand_worked_and_signed_zero():
    p = np.array([[0, 1, 3, 3, 10, -0.0]], dtype=np.float32)
    got = oracle.box_query(p, np.array([[1, -0.0, 11, np.nan]], np.float32),
                           np.array([[3, 0.0, 12, 5]], np.float32))
    assert [g.tolist() for g in got] == [[1, 2, 3], [0, 5], [], []]


def test_box_counts_agree_with_sorted_slabs():
    rng = np.random.default_rng(7)
    p = rng.integers(0, 50, size=(3, 2000)).astype(np.float32)
    lo = rng.integers(0, 50, size=(3, 40)).astype(np.float32)
    hi = lo + rng.integers(0, 30, size=(3, 40)).astype(np.float32)
    got = oracle.box_query(p, lo, hi)
    for i in range(40):
        keep = None
        for c in range(3):
            order = np.argsort(p[c], kind="stable")
            a = np.searchsorted(p[c][order], lo[c, i], side="left")
            b = np.searchsorted(p[c][order], hi[c, i], side="right")
            s = set(order[a:b].tolist())
            keep = s if keep is None else keep & s
        assert got[i].tolist() == sorted(keep)


@pytest.mark.parametrize("k", [1, 64])
def test_knn_fewer_points_than_k(k):
    p = np.array([[1.5, -2.0]], dtype=np.float32)
    idx, dist = oracle.knn(p, np.array([[0.0]], np.float32), k)
    assert idx[0, :min(k, 2)].tolist() == [0, 1][:k]
    assert (idx[0, 2:] == NONE).all() and np.isinf(dist[0, 2:]).all()
