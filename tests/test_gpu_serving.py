"""Serving on the GPU: requests built in a continuous-batching mix give the
same tree, bit for bit, as the same request built alone, and their leaf
lookups agree; a request that can never fit is rejected without stalling
the others."""
import sys
import threading
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("perm", "node_begin", "node_end", "node_child", "node_dim", "node_split", "node_leaf",
          "leaf_node", "leaf_offsets")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_requests(count, seed, lo_log2=10, hi_log2=17):
    import torch

    from paper_2201_08288_amd import synth
    out = []
    for k, (_, n, d) in enumerate(synth.poisson_requests(count, 1000.0, lo_log2, hi_log2,
                                                         seed=seed)):
        x = torch.from_numpy(synth.gmm(n, d, seed=seed, stream=k)).cuda()
        idx = np.random.default_rng(seed + k).integers(0, n, size=1024)
        out.append((x, x[:, torch.from_numpy(idx).cuda()].contiguous(), idx))
    torch.cuda.synchronize()
    return out


def test_served_results_equal_alone():
    import torch

    from paper_2201_08288_amd import kdtree, serve
    params = dict(leaf_size=64, num_subsets=64)
    reqs = make_requests(48, seed=31)
    log(f"case serving mix: {len(reqs)} requests, 3 workers")
    eng = serve.ServeEngine(params, cap_bytes=8 << 30, workers=3)
    done = []
    try:
        for k, (x, q, _) in enumerate(reqs):
            r = serve.Request(k, x, q, time.perf_counter())
            eng.submit(r)
            done.append(r)
            if k % 7 == 0:
                time.sleep(0.002)  # let batches form and overlap
        for r in done:
            assert r.event.wait(60), f"request {r.rid} did not finish"
    finally:
        eng.close()
    assert eng.batches < len(reqs), "no request was batched with another"
    log(f"batches {eng.batches}, sizes {eng.batch_sizes}")
    for r, (x, q, idx) in zip(done, reqs):
        assert r.status == kdtree.KD_OK, (r.rid, r.status)
        alone = kdtree.build(x, **params)
        la = kdtree.query_leaf(alone, q)
        torch.cuda.synchronize()
        a, b = alone.to_numpy(), r.tree.to_numpy()
        for f in ("num_nodes", "num_leaves", "depth", "point_levels", "status"):
            assert a[f] == b[f], (r.rid, f)
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (r.rid, f)
        assert torch.equal(la, r.leaves), r.rid
        # each lookup of a request's own point lands in the leaf holding it
        pos = np.argsort(a["perm"])[idx]
        leaf = np.searchsorted(a["leaf_offsets"], pos, side="right") - 1
        assert np.array_equal(r.leaves.cpu().numpy().view(np.uint32), leaf.astype(np.uint32))


def test_oversize_request_rejected_others_complete():
    from paper_2201_08288_amd import kdtree, serve
    params = dict(leaf_size=64, num_subsets=64)
    reqs = make_requests(6, seed=77, lo_log2=12, hi_log2=14)
    cap = 4 * max(serve.footprint_bytes(x.shape[1], x.shape[0], params, 1024) for x, _, _ in reqs)
    log(f"case serving admission: cap {cap} bytes")
    eng = serve.ServeEngine(params, cap_bytes=cap, workers=2)
    try:
        import torch
        big = torch.zeros((16, 1 << 22), device="cuda")
        rb = serve.Request(99, big, None, time.perf_counter())
        assert not eng.submit(rb)
        assert rb.event.is_set() and rb.status == kdtree.KD_ENOMEM
        done = []
        for k, (x, q, _) in enumerate(reqs):
            r = serve.Request(k, x, q, time.perf_counter())
            assert eng.submit(r)
            done.append(r)
        for r in done:
            assert r.event.wait(60) and r.status == kdtree.KD_OK, r.rid
        assert eng.used == 0
    finally:
        eng.close()


def test_inputs_still_being_written_when_submitted():
    """Points produced on the caller's stream right before submit (no host
    sync): the worker stream waits for them, so results equal the alone
    builds."""
    import torch

    from paper_2201_08288_amd import kdtree, serve
    print("case serving stream handoff", flush=True)
    params = dict(leaf_size=32, num_subsets=16)
    eng = serve.ServeEngine(params, cap_bytes=8 << 30, workers=2)
    gen = torch.Generator(device="cuda").manual_seed(5)
    reqs, data = [], []
    try:
        for k in range(12):
            x = torch.randn((3, 50000 + 1000 * k), generator=gen, device="cuda")
            x = x * 3.0 + 1.0  # more work queued on the caller's stream
            data.append(x)
            r = serve.Request(k, x, None, time.perf_counter())
            eng.submit(r)
            reqs.append(r)
        for r in reqs:
            assert r.event.wait(60)
    finally:
        eng.close()
    for r, x in zip(reqs, data):
        assert r.status == kdtree.KD_OK
        alone = kdtree.build(x, **params)
        torch.cuda.synchronize()
        a, b = alone.to_numpy(), r.tree.to_numpy()
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (r.rid, f)


def test_cancelled_request_leaves_others_unchanged():
    """One request of a mix is cancelled while queued and one while its
    batch builds; both end KD_ECANCELLED with their bytes freed, and every
    other request's tree equals its alone build."""
    import torch

    from paper_2201_08288_amd import kdtree, serve
    print("case serving cancellation", flush=True)
    params = dict(leaf_size=64, num_subsets=64)
    reqs = make_requests(24, seed=41, lo_log2=12, hi_log2=16)
    eng = serve.ServeEngine(params, cap_bytes=8 << 30, workers=1)
    done = []
    try:
        for k, (x, q, _) in enumerate(reqs):
            r = serve.Request(k, x, q, time.perf_counter())
            eng.submit(r)
            done.append(r)
            if k == 0:
                while done[0].state != "building":  # the first batch holds request 0 alone
                    time.sleep(0.0005)
                eng.cancel(done[0])
        eng.cancel(done[-1])  # still queued behind the first batch (one worker)
        for r in done:
            assert r.event.wait(60), r.rid
        assert eng.used == 0
    finally:
        eng.close()
    assert done[0].status == kdtree.KD_ECANCELLED and done[0].tree is None
    assert done[-1].status == kdtree.KD_ECANCELLED
    for r, (x, q, _) in list(zip(done, reqs))[1:-1]:
        assert r.status == kdtree.KD_OK, (r.rid, r.status)
        alone = kdtree.build(x, **params)
        torch.cuda.synchronize()
        a, b = alone.to_numpy(), r.tree.to_numpy()
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (r.rid, f)


def test_capacity_overflow_is_retried():
    """Node arrays far too small for the trees (node_capacity 16): every
    request comes back KD_ECAPACITY from the batch, is rebuilt alone with
    doubled capacity until it fits, and then equals the build with the
    default capacity."""
    import torch

    from paper_2201_08288_amd import kdtree, serve
    print("case serving capacity retry", flush=True)
    params = dict(leaf_size=64, num_subsets=64)
    reqs = make_requests(6, seed=43, lo_log2=12, hi_log2=14)
    eng = serve.ServeEngine(dict(params, node_capacity=16), cap_bytes=8 << 30, workers=2)
    done = []
    try:
        for k, (x, q, _) in enumerate(reqs):
            r = serve.Request(k, x, q, time.perf_counter())
            eng.submit(r)
            done.append(r)
        for r in done:
            assert r.event.wait(60), r.rid
    finally:
        eng.close()
    for r, (x, q, idx) in zip(done, reqs):
        assert r.status == kdtree.KD_OK and r.retries > 0, (r.rid, r.status, r.retries, r.error)
        alone = kdtree.build(x, **params)
        torch.cuda.synchronize()
        a, b = alone.to_numpy(), r.tree.to_numpy()
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (r.rid, f)
