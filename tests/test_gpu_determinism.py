"""Determinism: every workload and rule built three times gives the same
bytes (permutation, node arrays, leaf offsets, header and permuted points).
Atomics in the histogram, scatter and variance passes add integers, and
scans are fixed; a race would show up as a difference between runs."""
import numpy as np
import pytest

from paper_2201_08288_amd import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

FIELDS = ("perm", "node_begin", "node_end", "node_child", "node_dim", "node_split",
          "node_split_f", "node_leaf", "leaf_node", "leaf_offsets", "hdr", "points_out")


def _same(a, b):
    import torch
    h = a.header()
    assert h == b.header()
    size = {"leaf_node": h["num_leaves"], "leaf_offsets": h["num_leaves"] + 1}
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        if f.startswith("node_") or f.startswith("leaf_"):
            m = size.get(f, h["num_nodes"])
            x, y = x[:m], y[:m]
        assert torch.equal(x.view(torch.int32) if x.dtype == torch.float32 else x,
                           y.view(torch.int32) if y.dtype == torch.float32 else y), f


@pytest.mark.parametrize("workload", ["plain_n65536_d3", "scale_n2^24_d8", "hard_n2^26_d16"])
@pytest.mark.parametrize("rule", [0, 1, 2])
def test_three_builds_same_bytes(workload, rule):
    import torch

    from paper_2201_08288_amd import kdtree
    print(f"case determinism {workload} rule={rule}", flush=True)
    w = synth.WORKLOADS[workload]
    x = synth.generate(w["gen"], w["n"], w["d"])
    xt = torch.from_numpy(x).cuda()
    pool = None
    if w.get("pool_entries"):
        p = synth.dirichlet_pool(w["pool_entries"], w["num_subsets"], w["pool_alpha"])
        pool = torch.from_numpy(p.view(np.int32)).cuda()
    kw = dict(leaf_size=w["leaf_size"], num_subsets=w["num_subsets"], split_rule=rule,
              key_rule=1 if w["key"] == "maxvar" else 0, subset_pool=pool)
    first = kdtree.build(xt, **kw)
    for _ in range(2):
        again = kdtree.build(xt, **kw)
        torch.cuda.synchronize()
        _same(first, again)
        del again


def test_batched_three_runs_same_bytes():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case determinism batched 512 trees", flush=True)
    gen = torch.Generator(device="cuda").manual_seed(7)
    pts = [torch.randint(0, 1 << 24, (d, n), generator=gen, device="cuda").float() * 2.0 ** -24
           for n, d in synth.batched_shapes(512)]
    kw = dict(leaf_size=32, num_subsets=32)
    first = kdtree.build_batched(pts, **kw)
    for _ in range(2):
        again = kdtree.build_batched(pts, **kw)
        torch.cuda.synchronize()
        for a, b in zip(first, again):
            _same(a, b)
