"""Serving loop for tree builds: continuous batching over worker streams.

Requests (points already on the device) arrive at any time.  An admission
controller reserves each request's device footprint against a byte cap and
rejects requests that can never fit.  Each worker owns a HIP stream and, as
soon as it is free, takes every admitted request that is waiting and builds
them together with one kd_build_batched call (one set of level launches over
all of their cells); requests arriving meanwhile are picked up by the next
free worker, so builds from several batches overlap on the device.  After
its build each request runs its leaf lookups (kd_query_leaf) on the same
stream; the result is then handed back and the footprint released.

Every tree of a batch is bit-identical to a plain kd_build of that tree, so
a request's result does not depend on what it was batched with.
"""
import collections
import threading
import time

import torch

from . import kdtree


def footprint_bytes(n, d, leaf_size, num_queries=0):
    """Device bytes one request holds while in flight: input, output tree,
    permuted points and the build workspace (as sized by the library)."""
    prm = kdtree.make_params(leaf_size=leaf_size)
    cap, ws = kdtree.tree_bounds(n, d, prm)
    tree = 4 * n + cap * 4 * 9 + 4 * (cap + 1) + 32 + 4 * d * n
    return 4 * d * n + tree + ws + 8 * num_queries * d


class Request:
    __slots__ = ("rid", "points", "queries", "t_arrive", "t_admit", "t_done", "tree", "leaves",
                 "status", "bytes", "event", "ready")

    def __init__(self, rid, points, queries, t_arrive):
        self.rid, self.points, self.queries, self.t_arrive = rid, points, queries, t_arrive
        self.t_admit = self.t_done = None
        self.tree = self.leaves = None
        self.status = None
        self.bytes = 0
        self.event = threading.Event()
        self.ready = None  # device event: the inputs are complete on the submitting stream


class ServeEngine:
    """Continuous-batching build server on one GPU."""

    def __init__(self, params, cap_bytes=64 << 30, workers=2, max_batch=256, device="cuda:0"):
        self.params = dict(params)
        self.cap_bytes = cap_bytes
        self.max_batch = max_batch
        self.device = torch.device(device)
        self.used = 0
        self.lock = threading.Condition()
        self.waiting = collections.deque()   # admitted, not yet building
        self.pending = collections.deque()   # arrived, waiting for memory
        self.closed = False
        self.batches = 0
        self.batch_sizes = []
        self.workers = [threading.Thread(target=self._work, daemon=True) for _ in range(workers)]
        for w in self.workers:
            w.start()

    # -------------------------------------------------------------- admission
    def submit(self, req):
        if getattr(req.points, "is_cuda", False):
            # the build runs on a worker stream: it waits for the work that
            # produced the inputs on the caller's current stream
            req.ready = torch.cuda.Event()
            req.ready.record(torch.cuda.current_stream(req.points.device))
        d, n = req.points.shape
        nq = 0 if req.queries is None else req.queries.shape[1]
        req.bytes = footprint_bytes(n, d, self.params.get("leaf_size", 32), nq)
        with self.lock:
            if req.bytes > self.cap_bytes:
                req.status = kdtree.KD_ENOMEM
                req.t_done = time.perf_counter()
                req.event.set()
                return False
            self.pending.append(req)
            self._admit_locked()
            self.lock.notify_all()
        return True

    def _admit_locked(self):
        # first come, first served: a large request at the head waits for memory
        while self.pending and self.used + self.pending[0].bytes <= self.cap_bytes:
            r = self.pending.popleft()
            self.used += r.bytes
            r.t_admit = time.perf_counter()
            self.waiting.append(r)

    def _release(self, reqs):
        with self.lock:
            for r in reqs:
                self.used -= r.bytes
            self._admit_locked()
            self.lock.notify_all()

    # -------------------------------------------------------------- workers
    def _make_stream(self):
        torch.cuda.set_device(self.device)
        return torch.cuda.Stream(device=self.device)

    def _run_batch(self, batch, stream):
        """One batched build of every request of the batch, then each
        request's lookups, all on this worker's stream."""
        with torch.cuda.stream(stream):
            for r in batch:
                if r.ready is not None:
                    stream.wait_event(r.ready)
            trees = kdtree.build_batched([r.points for r in batch], stream=stream, **self.params)
            for r, t in zip(batch, trees):
                r.tree = t
                if r.queries is not None:
                    r.leaves = kdtree.query_leaf(t, r.queries, stream=stream)
        stream.synchronize()

    def _work(self):
        stream = self._make_stream()
        while True:
            with self.lock:
                while not self.waiting and not self.closed:
                    self.lock.wait()
                if self.closed and not self.waiting:
                    return
                batch = []
                while self.waiting and len(batch) < self.max_batch:
                    batch.append(self.waiting.popleft())
                self.batches += 1
                self.batch_sizes.append(len(batch))
            try:
                self._run_batch(batch, stream)
                for r in batch:
                    r.status = kdtree.KD_OK
            except kdtree.KDError as e:
                for r in batch:
                    r.status = e.status
            now = time.perf_counter()
            for r in batch:
                r.t_done = now
            self._release(batch)
            for r in batch:
                r.event.set()

    def close(self):
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        for w in self.workers:
            w.join()


def run_poisson(engine, requests, rate, seed=0):
    """Submit (points, queries) pairs with exponential gaps of mean 1/rate;
    returns the Request objects after all have completed."""
    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=len(requests))
    out = []
    t0 = time.perf_counter()
    t_next = t0
    for k, (pts, q) in enumerate(requests):
        t_next += gaps[k]
        while True:
            now = time.perf_counter()
            if now >= t_next:
                break
            time.sleep(min(t_next - now, 0.001))
        r = Request(k, pts, q, t_next)
        engine.submit(r)
        out.append(r)
    for r in out:
        r.event.wait()
    return out


def latency_stats(reqs):
    import numpy as np
    lat = np.array([r.t_done - r.t_arrive for r in reqs if r.status == kdtree.KD_OK])
    pts = sum(r.points.shape[1] for r in reqs if r.status == kdtree.KD_OK)
    span = max(r.t_done for r in reqs) - min(r.t_arrive for r in reqs)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "requests": len(lat), "points_per_s": pts / span, "span_s": span}
