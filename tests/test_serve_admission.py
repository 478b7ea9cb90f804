"""Host logic of the serving loop (no GPU): admission against the byte cap,
first-come-first-served order, rejection of requests that can never fit,
and batches formed from whatever is waiting when a worker frees up."""
import threading
import time

import pytest

from paper_2201_08288_amd import kdtree, serve


class FakePoints:
    def __init__(self, d, n):
        self.shape = (d, n)


class HostEngine(serve.ServeEngine):
    """The serving loop with the device work replaced by a sleep, recording
    the bytes in flight."""

    def __init__(self, *a, work_s=0.01, **kw):
        self.work_s = work_s
        self.peak = 0
        self.order = []
        self.rec = threading.Lock()
        super().__init__(*a, **kw)

    def _make_stream(self):
        return None

    def _run_batch(self, batch, stream):
        with self.rec:
            self.peak = max(self.peak, self.used)
            self.order.extend(r.rid for r in batch)
        time.sleep(self.work_s)
        return [kdtree.KD_OK] * len(batch)


class FailingEngine(HostEngine):
    """Device work that raises something other than a library error."""

    def _run_batch(self, batch, stream):
        time.sleep(self.work_s)
        raise RuntimeError("out of device memory (simulated)")


def fp(n, d, **params):
    return serve.footprint_bytes(n, d, dict(dict(leaf_size=32), **params))


def test_footprint_grows_with_size():
    assert fp(1 << 12, 3) < fp(1 << 13, 3) < fp(1 << 13, 16)
    assert fp(1 << 20, 3) > 4 * 3 * (1 << 20) * 2


def test_footprint_follows_the_build_parameters():
    """The workspace the library asks for grows with the split rule, the
    subset count and the largest-variance key's per-cell sums; admission must
    count it (the library's own bound, not a default-parameter one)."""
    n, d = 1 << 20, 16
    exact = fp(n, d)
    assert fp(n, d, split_rule=kdtree.SPLIT_FOURIER) > exact
    assert fp(n, d, split_rule=kdtree.SPLIT_SUBSET, num_subsets=256) > \
        fp(n, d, split_rule=kdtree.SPLIT_SUBSET, num_subsets=4) > exact
    assert fp(n, d, key_rule=kdtree.KEY_MAXVAR) > exact
    for prm in (dict(split_rule=kdtree.SPLIT_FOURIER), dict(key_rule=kdtree.KEY_MAXVAR),
                dict(split_rule=kdtree.SPLIT_SUBSET, num_subsets=64)):
        full = dict(leaf_size=32, **prm)
        cap, ws = kdtree.tree_bounds(n, d, kdtree.make_params(**full))
        assert fp(n, d, **prm) >= ws + 8 * d * n


def test_cap_respected_and_fifo():
    sizes = [(1 << 12, 3)] * 20 + [(1 << 14, 8)] * 5
    cap = 3 * fp(1 << 14, 8)
    eng = HostEngine({"leaf_size": 32}, cap_bytes=cap, workers=3, work_s=0.005)
    reqs = []
    try:
        for k, (n, d) in enumerate(sizes):
            r = serve.Request(k, FakePoints(d, n), None, time.perf_counter())
            assert eng.submit(r)
            reqs.append(r)
        for r in reqs:
            assert r.event.wait(10)
    finally:
        eng.close()
    assert all(r.status == kdtree.KD_OK for r in reqs)
    assert eng.peak <= cap
    assert eng.used == 0
    # admission is first come, first served
    assert sorted(eng.order) == list(range(len(sizes)))
    admit = sorted(reqs, key=lambda r: r.t_admit)
    assert [r.rid for r in admit] == list(range(len(sizes)))


def test_never_fitting_request_rejected():
    eng = HostEngine({"leaf_size": 32}, cap_bytes=fp(1 << 12, 3) * 2, workers=1)
    try:
        r = serve.Request(0, FakePoints(16, 1 << 20), None, time.perf_counter())
        assert not eng.submit(r)
        assert r.status == kdtree.KD_ENOMEM and r.event.is_set()
        ok = serve.Request(1, FakePoints(3, 1 << 12), None, time.perf_counter())
        assert eng.submit(ok)
        assert ok.event.wait(10) and ok.status == kdtree.KD_OK
    finally:
        eng.close()


def test_requests_arriving_during_work_are_batched():
    eng = HostEngine({"leaf_size": 32}, cap_bytes=1 << 40, workers=1, work_s=0.05)
    reqs = []
    try:
        for k in range(9):
            r = serve.Request(k, FakePoints(3, 1 << 12), None, time.perf_counter())
            eng.submit(r)
            reqs.append(r)
        for r in reqs:
            assert r.event.wait(10)
    finally:
        eng.close()
    # the first request starts alone; the rest wait and go together
    assert eng.batch_sizes[0] >= 1 and len(eng.batch_sizes) < 9
    assert sum(eng.batch_sizes) == 9


def test_latency_stats():
    reqs = []
    for k in range(100):
        r = serve.Request(k, FakePoints(3, 1000), None, float(k))
        r.t_done = k + 0.001 * (k + 1)
        r.status = kdtree.KD_OK
        reqs.append(r)
    st = serve.latency_stats(reqs)
    assert st["requests"] == 100
    assert 0.049 <= st["p50_ms"] / 1e3 <= 0.052
    assert st["p99_ms"] <= 100.0 + 1e-9


def test_worker_exception_releases_and_wakes():
    """An unexpected failure of a batch (not a library status) ends every
    request of the batch with KD_EDEVICE and the error text, frees its bytes
    and lets later requests run."""
    eng = FailingEngine({"leaf_size": 32}, cap_bytes=1 << 40, workers=1, work_s=0.01)
    try:
        reqs = [serve.Request(k, FakePoints(3, 1 << 12), None, time.perf_counter())
                for k in range(5)]
        for r in reqs:
            eng.submit(r)
        for r in reqs:
            assert r.event.wait(10)
            assert r.status == kdtree.KD_EDEVICE and "simulated" in r.error
        assert eng.used == 0
    finally:
        eng.close()


def test_cancel_before_and_during_build():
    """Cancelled while queued: leaves at once, bytes freed.  Cancelled while
    its batch builds: the batch finishes, the request ends KD_ECANCELLED and
    its bytes are freed; other requests are unaffected."""
    size = fp(1 << 12, 3)
    eng = HostEngine({"leaf_size": 32}, cap_bytes=2 * size, workers=1, work_s=0.2)
    try:
        reqs = [serve.Request(k, FakePoints(3, 1 << 12), None, time.perf_counter())
                for k in range(4)]
        assert eng.submit(reqs[0])
        while reqs[0].state != "building":
            time.sleep(0.001)
        for r in reqs[1:]:
            assert eng.submit(r)
        # request 0 builds; 1 is admitted and waits; 2, 3 wait for memory
        assert reqs[0].state == "building"
        assert reqs[1].state == "waiting" and reqs[2].state == "pending"
        assert eng.cancel(reqs[2]) and reqs[2].status == kdtree.KD_ECANCELLED
        assert eng.cancel(reqs[1]) and reqs[1].status == kdtree.KD_ECANCELLED
        # the freed bytes admit request 3 at once
        assert reqs[3].state == "waiting" and eng.used == 2 * size
        assert eng.cancel(reqs[0])
        for r in reqs:
            assert r.event.wait(10)
        assert reqs[0].status == kdtree.KD_ECANCELLED
        assert reqs[3].status == kdtree.KD_OK
        assert not eng.cancel(reqs[3])  # already finished
        assert eng.used == 0
    finally:
        eng.close()
