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


def footprint_bytes(n, d, params, num_queries=0):
    """Device bytes one request holds while in flight: input, output tree,
    permuted points and the build workspace, as the library sizes them for
    these build parameters (split rule, subsets, key rule, leaf size,
    node capacity)."""
    prm = kdtree.make_params(**params)
    cap, ws = kdtree.tree_bounds(n, d, prm)
    tree = 4 * n + cap * 4 * 9 + 4 * (cap + 1) + 32 + 4 * d * n
    return 4 * d * n + tree + ws + 8 * num_queries * d


class Request:
    __slots__ = ("rid", "points", "queries", "t_arrive", "t_admit", "t_done", "tree", "leaves",
                 "status", "bytes", "event", "ready", "state", "cancel_asked", "retries", "error")

    def __init__(self, rid, points, queries, t_arrive):
        self.rid, self.points, self.queries, self.t_arrive = rid, points, queries, t_arrive
        self.t_admit = self.t_done = None
        self.tree = self.leaves = None
        self.status = None
        self.bytes = 0
        self.event = threading.Event()
        self.ready = None  # device event: the inputs are complete on the submitting stream
        self.state = "new"  # new -> pending -> waiting -> building -> done
        self.cancel_asked = False
        self.retries = 0    # rebuilds with larger node arrays after KD_ECAPACITY
        self.error = None   # text of an unexpected failure of its batch


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
        req.bytes = footprint_bytes(n, d, self.params, nq)
        with self.lock:
            if req.bytes > self.cap_bytes:
                self._finish_locked(req, kdtree.KD_ENOMEM)
                return False
            req.state = "pending"
            self.pending.append(req)
            self._admit_locked()
            self.lock.notify_all()
        return True

    def cancel(self, req):
        """Withdraw a request.  Not yet building: it leaves the queues at once
        and its reserved bytes are freed.  Building: its batch runs to the end
        (the other requests' results do not depend on it), then its result is
        dropped and its bytes freed with the batch.  Either way it ends with
        status KD_ECANCELLED.  Returns False if it had already finished."""
        with self.lock:
            if req.state == "done":
                return False
            req.cancel_asked = True
            if req.state == "pending":
                self.pending.remove(req)
                self._finish_locked(req, kdtree.KD_ECANCELLED)
            elif req.state == "waiting":
                self.waiting.remove(req)
                self.used -= req.bytes
                self._finish_locked(req, kdtree.KD_ECANCELLED)
                self._admit_locked()
            self.lock.notify_all()
        return True

    def _finish_locked(self, req, status):
        req.status = status
        req.state = "done"
        req.t_done = time.perf_counter()
        if status != kdtree.KD_OK:
            req.tree = req.leaves = None
        req.event.set()

    def _admit_locked(self):
        # first come, first served: a large request at the head waits for memory
        while self.pending and self.used + self.pending[0].bytes <= self.cap_bytes:
            r = self.pending.popleft()
            self.used += r.bytes
            r.t_admit = time.perf_counter()
            r.state = "waiting"
            self.waiting.append(r)

    def _release(self, reqs, statuses):
        with self.lock:
            for r, st in zip(reqs, statuses):
                self.used -= r.bytes
                self._finish_locked(r, kdtree.KD_ECANCELLED if r.cancel_asked else st)
            self._admit_locked()
            self.lock.notify_all()

    # -------------------------------------------------------------- workers
    def _make_stream(self):
        torch.cuda.set_device(self.device)
        return torch.cuda.Stream(device=self.device)

    def _run_batch(self, batch, stream):
        """One batched build of every request of the batch, then each
        request's lookups, all on this worker's stream.  Returns each
        request's status: a tree whose node arrays were too small (header
        status KD_ECAPACITY) is rebuilt alone with twice the node capacity,
        up to the most nodes a tree of its size can have (2n - 1)."""
        with torch.cuda.stream(stream):
            for r in batch:
                if r.ready is not None:
                    stream.wait_event(r.ready)
            trees = kdtree.build_batched([r.points for r in batch], stream=stream, **self.params)
            for r, t in zip(batch, trees):
                r.tree = t
        stream.synchronize()
        statuses = []
        for r in batch:
            h = r.tree.header()
            while h["status"] == kdtree.KD_ECAPACITY and r.tree.cap < 2 * r.points.shape[1] + 64:
                r.retries += 1
                prm = dict(self.params, node_capacity=2 * r.tree.cap)
                with torch.cuda.stream(stream):
                    r.tree = kdtree.build(r.points, stream=stream, **prm)
                stream.synchronize()
                h = r.tree.header()
            statuses.append(h["status"])
        with torch.cuda.stream(stream):
            for r, st in zip(batch, statuses):
                if st == kdtree.KD_OK and r.queries is not None:
                    r.leaves = kdtree.query_leaf(r.tree, r.queries, stream=stream)
        stream.synchronize()
        return statuses

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
                    r = self.waiting.popleft()
                    r.state = "building"
                    batch.append(r)
                self.batches += 1
                self.batch_sizes.append(len(batch))
            statuses = [kdtree.KD_EDEVICE] * len(batch)
            try:
                statuses = self._run_batch(batch, stream)
            except kdtree.KDError as e:
                statuses = [e.status] * len(batch)
            except Exception as e:  # noqa: BLE001 -- every request must end
                for r in batch:
                    r.error = f"{type(e).__name__}: {e}"
            finally:
                # whatever happened, the batch's bytes are released and every
                # waiter is woken
                self._release(batch, statuses)

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
