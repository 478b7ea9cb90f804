"""kd_build_noalloc (the library's fixed per-device workspace, no
allocation) against kd_build with a caller's workspace: two calls in a row,
the second on a smaller input, each tree equal bit for bit to kd_build's and
to the oracle's; a build too large for the fixed workspace is rejected
before any work is enqueued."""
import numpy as np
import pytest

import oracle
from paper_2201_08288_amd import synth
from tests.gpu_common import HDR_KEYS, TREE_KEYS, assert_same_tree

pytestmark = pytest.mark.gpu


def test_noalloc_equals_build_two_calls_second_smaller():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case no-alloc build: two calls, second smaller", flush=True)
    cases = [(synth.student_t_grid(400_000, 4, seed=91), dict(split_rule=1, key_rule=1)),
             (synth.gmm(90_000, 3, seed=92), dict(split_rule=0, key_rule=0))]
    for x, extra in cases:
        kw = dict(leaf_size=32, num_subsets=16, **extra)
        xt = torch.from_numpy(x).cuda()
        ref = kdtree.build(xt, **kw)
        na = kdtree.KDTree(xt.shape[1], xt.shape[0], ref.cap, xt.device)
        kdtree.build_noalloc(xt, na, **kw)
        torch.cuda.synchronize()
        a, b = ref.to_numpy(), na.to_numpy()
        for k in HDR_KEYS:
            assert a[k] == b[k], k
        for k in TREE_KEYS + ("points_out",):
            assert np.array_equal(np.asarray(a[k]).view(np.uint32),
                                  np.asarray(b[k]).view(np.uint32)), k
        assert_same_tree(b, oracle.build_tree(x, **kw), x)


def test_noalloc_rejects_a_build_beyond_the_scratch():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case no-alloc build: too large", flush=True)
    n, d = 1 << 21, 8
    cap, ws = kdtree.tree_bounds(n, d, kdtree.make_params(leaf_size=32))
    assert ws > kdtree.NOALLOC_SCRATCH_BYTES
    xt = torch.zeros((d, n), device="cuda")
    t = kdtree.KDTree(n, d, cap, xt.device)
    t.hdr.fill_(-7)
    with pytest.raises(kdtree.KDError) as e:
        kdtree.build_noalloc(xt, t, leaf_size=32)
    assert e.value.status == kdtree.KD_ENOMEM
    torch.cuda.synchronize()
    assert int(t.hdr[0].item()) == -7  # nothing was enqueued
