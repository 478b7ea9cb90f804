"""kd_build and kd_build_batched are stream-ordered: they enqueue every level
and return without waiting for the device, so the host gets control back
while earlier work on the stream is still running, and a build can be
captured in a graph and replayed.  Every result is compared with the oracle
bit for bit."""
import time

import numpy as np
import pytest

import oracle
from paper_2201_08288_amd import synth
from tests.gpu_common import assert_same_tree

pytestmark = pytest.mark.gpu

SLEEP_CYCLES = 200_000_000  # a spin kernel of this many GPU clocks: tens of milliseconds


@pytest.mark.parametrize("rule", [0, 1, 2])
def test_build_returns_before_the_stream_completes(rule):
    import torch

    from paper_2201_08288_amd import kdtree
    print(f"case stream-ordered build rule={rule}", flush=True)
    x = synth.gmm(300_000, 5, seed=11 + rule)
    kw = dict(leaf_size=32, num_subsets=16, split_rule=rule)
    xt = torch.from_numpy(x).cuda()
    warm = kdtree.build(xt, **kw)  # workspace and output arrays, and the library loaded
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda._sleep(SLEEP_CYCLES)  # keeps the stream busy
        t0 = time.perf_counter()
        tree = kdtree.build(xt, workspace=warm.workspace, tree=warm, stream=s, **kw)
        t_call = time.perf_counter() - t0
        busy = not s.query()
    assert busy, "kd_build waited for the stream"
    s.synchronize()
    print(f"kd_build returned after {1e3 * t_call:.2f} ms with the stream still busy", flush=True)
    assert_same_tree(tree.to_numpy(), oracle.build_tree(x, **kw), x)


def test_batched_returns_before_the_stream_completes():
    import torch

    from paper_2201_08288_amd import kdtree
    print("case stream-ordered batched build", flush=True)
    xs = [synth.uniform24(n, d, seed=60 + k) for k, (n, d) in
          enumerate([(5000, 2), (70000, 3), (300, 8), (120000, 32), (4097, 3)])]
    kw = dict(leaf_size=32, num_subsets=8)
    dev = [torch.from_numpy(x).cuda() for x in xs]
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda._sleep(SLEEP_CYCLES)
        trees = kdtree.build_batched(dev, stream=s, **kw)
        busy = not s.query()
    assert busy, "kd_build_batched waited for the stream"
    s.synchronize()
    for x, t, o in zip(xs, trees, oracle.build_trees(xs, **kw)):
        assert_same_tree(t.to_numpy(), o, x)


@pytest.mark.parametrize("rule,key", [(0, 0), (1, 0), (2, 1)])
def test_graph_capture_and_replay(rule, key):
    """One kd_build captured in a graph; the input is rewritten between
    replays (eager work and synchronizations in between), and every replay
    must equal the eager build and the oracle on that input."""
    import torch

    from paper_2201_08288_amd import kdtree
    print(f"case graph capture rule={rule} key={key}", flush=True)
    kw = dict(leaf_size=40, num_subsets=8, split_rule=rule, key_rule=key)
    inputs = [synth.student_t_grid(150_000, 4, seed=70 + k) for k in range(3)]
    xt = torch.from_numpy(inputs[0]).cuda()
    eager = kdtree.build(xt, **kw)  # allocations happen outside the graph
    torch.cuda.synchronize()
    ws = eager.workspace
    out = kdtree.KDTree(xt.shape[1], xt.shape[0], eager.cap, xt.device)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        kdtree.build(xt, workspace=ws, tree=out, **kw)
    torch.cuda.synchronize()
    for rep in range(3):
        x = inputs[rep % len(inputs)]
        xt.copy_(torch.from_numpy(x).cuda())
        y = torch.ones(1 << 20, device="cuda") * 2.0  # unrelated eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(y.sum().item()) == float(2 << 20)
        got = out.to_numpy()
        ref = kdtree.build(xt, **kw)
        torch.cuda.synchronize()
        want = ref.to_numpy()
        for k in ("perm", "node_child", "node_dim", "node_split", "leaf_offsets", "points_out"):
            assert np.array_equal(np.asarray(got[k]).view(np.uint32),
                                  np.asarray(want[k]).view(np.uint32)), (rep, k)
        assert_same_tree(got, oracle.build_tree(x, **kw), x)
