"""Launch shapes and digit widths never change the tree: builds under every
setting the tuner tries are bit-identical to each other and to the oracle,
and kd_autotune keeps one of them."""
import numpy as np
import pytest

from paper_2201_08288_amd import synth
from tests.gpu_common import assert_same_tree, gpu_tree, oracle_tree

pytestmark = pytest.mark.gpu

SHAPES = [dict(), dict(hist_blocks=512), dict(hist_blocks=1), dict(scatter_blocks=1024),
          dict(scatter_blocks=1), dict(small_blocks=2048), dict(small_blocks=1),
          dict(hist_blocks=3, scatter_blocks=7, small_blocks=5), dict(digit_bits=8),
          dict(digit_bits=8, hist_blocks=5, scatter_blocks=3)]


@pytest.mark.parametrize("rule,key", [(0, 0), (1, 0), (2, 1)])
def test_every_launch_shape_builds_the_same_tree(rule, key):
    from paper_2201_08288_amd import kdtree
    x = synth.gmm(70000, 3, seed=21 + rule)
    kw = dict(leaf_size=16, num_subsets=8, split_rule=rule, key_rule=key)
    o = oracle_tree(x, **kw)
    before = kdtree.get_tuning()
    try:
        for shape in SHAPES:
            print(f"case tuning rule={rule} key={key} {shape}", flush=True)
            kdtree.set_tuning(**shape)
            assert_same_tree(gpu_tree(x, **kw)[1], o, x)
    finally:
        kdtree.set_tuning(**before)


def test_autotune_keeps_a_valid_shape():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case autotune", flush=True)
    x = synth.uniform24(1 << 18, 4, seed=4)
    before = kdtree.get_tuning()
    try:
        best = kdtree.autotune(torch.from_numpy(x).cuda(), leaf_size=32, num_subsets=16)
        assert kdtree.get_tuning() == best
        kw = dict(leaf_size=32, num_subsets=16)
        assert_same_tree(gpu_tree(x, **kw)[1], oracle_tree(x, **kw), x)
    finally:
        kdtree.set_tuning(**before)
