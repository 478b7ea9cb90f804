"""GPU parity of the global single-pass construction against the oracle:
identical int64 statistics, bit-identical fp64 medians, identical leaf
counts; plus the map-reduce property and the §5.1 accuracy panel at scale."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def unit_points(n, p, seed, kind="uniform"):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.random((p, n)).astype(np.float32).clip(2.0 ** -24, 1 - 2.0 ** -24)
    if kind == "ties":
        return (rng.integers(1, 64, size=(p, n)) / 64.0).astype(np.float32)
    if kind == "outside":  # not in (0,1): no clamping on either side, same results
        return (rng.random((p, n)) * 2.0 - 0.5).astype(np.float32)
    from scipy.stats import norm

    from paper_2201_08288_amd import synth
    x = synth.corr_normal(n, p, rho=0.5, seed=seed)
    return np.clip(norm.cdf(x), 2.0 ** -24, 1 - 2.0 ** -24).astype(np.float32)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("n,J,depth,kind", [(1, 15, 3, "uniform"), (1000, 3, 5, "uniform"),
                                            (70001, 15, 6, "normal"), (20000, 7, 8, "ties"),
                                            (5000, 15, 4, "outside")])
def test_global_matches_oracle(p, n, J, depth, kind):
    import torch

    from paper_2201_08288_amd import kdtree
    print(f"case global p={p} n={n} J={J} depth={depth} {kind}", flush=True)
    x = unit_points(n, p, seed=n + p, kind=kind)
    xt = torch.from_numpy(x).cuda()
    C = kdtree.global_moments(xt, J)
    med = kdtree.global_solve(C, p, J, depth)
    cnt = kdtree.global_counts(xt, med, depth)
    o = oracle.global_build(x, J=J, depth=depth)
    assert np.array_equal(C.cpu().numpy(), o["moments"])
    assert np.array_equal(med.cpu().numpy().view(np.uint64), o["medians"].view(np.uint64))
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint64), o["counts"])


def test_global_moments_add_over_subsets():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case global subsets", flush=True)
    x = torch.from_numpy(unit_points(300001, 3, seed=5)).cuda()
    whole = kdtree.global_moments(x, 15)
    acc = torch.zeros_like(whole)
    for a, b in ((0, 1), (1, 99999), (99999, 300001)):
        kdtree.global_moments(x[:, a:b], 15, moments=acc)
    assert torch.equal(whole, acc)
    assert int(whole[0].item()) == 300001 * 2 ** 30


@pytest.mark.slow
def test_global_at_scale_and_paper_panel():
    """n = 2^24 trivariate normal (rho = 0.5) through the normal CDF: the
    exact count statistic, the solve and the counts against the oracle on the
    GPU's statistics, and the cell-count spread against §5.1's panel."""
    import json
    import os

    import torch

    from paper_2201_08288_amd import kdtree
    print("case global scale n=2^24", flush=True)
    n, depth = 1 << 24, 6
    x = unit_points(n, 3, seed=21, kind="normal")
    xt = torch.from_numpy(x).cuda()
    C = kdtree.global_moments(xt, 15)
    med = kdtree.global_solve(C, 3, 15, depth)
    cnt = kdtree.global_counts(xt, med, depth).cpu().numpy()
    Cn = C.cpu().numpy()
    assert Cn[0] == n * 2 ** 30
    assert np.array_equal(med.cpu().numpy().view(np.uint64),
                          oracle.global_solve(Cn, 3, 15, depth).view(np.uint64))
    assert np.array_equal(cnt.astype(np.uint64), oracle.global_counts(x, med.cpu().numpy(), depth))
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_accuracy_panel.json")) as f:
        g = json.load(f)
    rel = np.log2(cnt / (n / 2 ** depth))
    q1, q3 = np.percentile(rel, [25, 75])
    print(f"spread log2: min {rel.min():.4f} max {rel.max():.4f} iqr {q1:.4f} {q3:.4f}", flush=True)
    assert -0.03 <= q1 and q3 <= 0.03
    assert rel.min() > -0.1 and rel.max() < 0.1
