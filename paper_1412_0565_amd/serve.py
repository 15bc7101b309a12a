"""Continuous-batching Fiedler server on one GPU.

Requests (a graph and its id) arrive at any time.  The server

* admits a request when its device-memory footprint fits the budget next to
  everything already resident or in flight (admission by HBM footprint);
* builds its hierarchy (``cmg_setup``) on a setup thread while the solve
  thread solves earlier requests.  Both issue their work to one HIP stream:
  a solve's grid levels wait at grid barriers for all their workgroups, and
  setup kernels from a second stream could hold compute units long enough
  to exhaust the barrier's bounded wait.  The host-side work of the two
  threads overlaps; the device runs their kernels in issue order;
* solves the ready requests in packed batches (``cmg_fiedler_batch``), so
  requests that arrive while a batch is on the GPU join a following one
  (continuous batching, not a queue).  A batch returns when its longest
  solve ends, so batches are formed by expected cost: the cheapest ready
  request first (shortest job first, with requests that waited longer than
  ``max_wait_s`` taken first), then others of at most ``cost_ratio`` times
  its cost.  The cost of a graph is its last measured solve time, or an
  estimate from its size before the first;
* keeps hierarchies resident, keyed by graph id, and evicts the least
  recently used ones that are not in use when memory is needed, so a repeat
  graph skips the setup phase;
* honours a per-request deadline (``timeout_s``) and ``cancel``: a request
  that expires or is cancelled before its batch starts is dropped with
  status "timeout" or "cancelled"; one already on the GPU completes;
* records arrival, admission, setup, and completion times per request.

The solve results equal those of a solo ``cmg_fiedler`` bit for bit: the
batch runs the same kernels with the same workgroup counts per graph.

The device work goes through a backend object (``CmgBackend`` for the GPU);
tests drive the scheduler with a fake backend on the CPU.
"""
from __future__ import annotations

import collections
import ctypes as C
import dataclasses
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    graph_id: object
    n: int
    row_ptr: object
    col: object
    w: object
    precision: int = 0
    t_arrive: float = 0.0
    t_admit: float = 0.0
    t_ready: float = 0.0
    t_done: float = 0.0
    lam: float = float("nan")
    x: np.ndarray | None = None
    status: str = "queued"
    error: str = ""
    resident_hit: bool = False
    timeout_s: float | None = None  # deadline after arrival; None: none
    cancelled: bool = False
    event: threading.Event = dataclasses.field(default_factory=threading.Event)

    def expired(self, now: float) -> bool:
        return self.timeout_s is not None and now - self.t_arrive > self.timeout_s

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


def estimate_footprint(n: int, nnz: int) -> int:
    """Upper estimate of the device bytes a hierarchy needs while it is
    built: the level-0 copy (12 B/entry, 4 B/row), coarse levels (at most
    about 0.8x level 0 on meshes), two refinement vectors per level, and the
    setup scratch (radix-sort double buffer of 16 B/entry keys+values, head
    flags and offsets)."""
    level0 = 12 * nnz + 4 * (n + 1)
    hierarchy = int(1.8 * level0) + 2 * 8 * 2 * n
    scratch = 40 * nnz + 48 * n
    return hierarchy + scratch + (1 << 20)


class CmgBackend:
    """GPU backend: libcmg through the C-ABI binding."""

    def __init__(self, device: int = 0):
        import torch

        from . import cmg

        self.cmg = cmg
        self.torch = torch
        torch.cuda.set_device(device)
        # one device stream for both: a setup's kernels on a second stream
        # can keep a solve's grid-barrier workgroups from all becoming
        # resident (setup and solve still overlap on the host threads)
        self.setup_stream = torch.cuda.Stream()
        self.solve_stream = self.setup_stream
        self.alloc = cmg.torch_allocator()

    def setup(self, req: Request):
        """Returns (handle, resident bytes)."""
        cmg = self.cmg
        with self.torch.cuda.stream(self.setup_stream):
            opt = cmg.cmg_options_default(precision=req.precision, allocator=C.pointer(self.alloc),
                                          stream=C.c_void_p(self.setup_stream.cuda_stream))
            h = cmg.cmg_setup(req.n, req.row_ptr, req.col, req.w, opt)
        cmg.cmg_set_stream(h, self.solve_stream)
        return h, cmg.cmg_footprint(h)

    def solve(self, handles, ns):
        cmg = self.cmg
        xs = [np.zeros(n) for n in ns]
        lams, status = cmg.cmg_fiedler_batch(handles, xs)
        return lams, xs

    def free(self, h):
        self.cmg.cmg_free(h)


def estimate_cost(n: int, nnz: int) -> float:
    """Seconds a first solve of an unseen graph is expected to take: a
    launch floor plus streaming its levels a few hundred times (an upper
    estimate; measured times replace it)."""
    return 2e-3 + 400 * 16.0 * nnz / 2e12


class Server:
    def __init__(self, backend, budget_bytes: int, max_batch: int = 64, resident_cap: int | None = None,
                 cost_ratio: float = 2.0, max_wait_s: float = 0.5, policy: str = "cost"):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.resident_cap = resident_cap
        self.cost_ratio = cost_ratio
        self.max_wait_s = max_wait_s
        self.policy = policy                   # "cost" (cost-aware batches) or "fifo" (arrival order)
        self.cost = {}                         # graph_id -> last measured solve seconds
        self.evictions = 0
        self.lock = threading.Condition()
        self.pending = collections.deque()     # arrived, not admitted
        self.setup_q = collections.deque()     # admitted, waiting for setup
        self.ready = collections.deque()       # hierarchy built, waiting for a batch
        self.resident = collections.OrderedDict()  # graph_id -> [handle, bytes, users]
        self.reserved = 0                      # bytes reserved by admitted requests in setup
        self.used = 0                          # bytes of resident hierarchies
        self.done = []
        self.batches = []                      # sizes of the solved batches
        self.peak = 0
        self.stop = False
        self.threads = [threading.Thread(target=self._setup_loop, daemon=True),
                        threading.Thread(target=self._solve_loop, daemon=True)]
        for t in self.threads:
            t.start()

    # ---------------------------------------------------------------- API
    def submit(self, req: Request) -> Request:
        with self.lock:
            req.t_arrive = req.t_arrive or time.perf_counter()
            self.pending.append(req)
            self._admit()
            self.lock.notify_all()
        return req

    def cancel(self, req: Request) -> None:
        """Drop `req` unless its batch has started (then it completes)."""
        with self.lock:
            req.cancelled = True
            self._drop_stale(time.perf_counter())
            self.lock.notify_all()

    def close(self):
        with self.lock:
            self.stop = True
            self.lock.notify_all()
        for t in self.threads:
            t.join()
        for gid, (h, b, users) in list(self.resident.items()):
            self.backend.free(h)
        self.resident.clear()

    # ---------------------------------------------------------- internals
    def _finish(self, req: Request, status: str, error: str = "") -> None:
        req.status = status
        req.error = error
        req.t_done = time.perf_counter()
        req.event.set()
        self.done.append(req)

    def _drop_stale(self, now: float) -> None:
        """Cancelled or expired requests leave the pending and ready queues
        (caller holds the lock); a ready one gives back its residency use."""
        for q in (self.pending, self.ready):
            keep = collections.deque()
            for req in q:
                if req.cancelled or req.expired(now):
                    if q is self.ready:
                        ent = self.resident.get(req.graph_id)
                        if ent is not None:
                            ent[2] -= 1
                    self._finish(req, "cancelled" if req.cancelled else "timeout")
                else:
                    keep.append(req)
            q.clear()
            q.extend(keep)

    def _req_cost(self, req: Request) -> float:
        c = self.cost.get(req.graph_id)
        return c if c is not None else estimate_cost(req.n, int(req.col.shape[0]))

    def _pick_batch(self, now: float):
        """Cost-aware batch (caller holds the lock): the cheapest ready
        request, or the longest-waiting one past max_wait_s, then other
        ready requests of at most cost_ratio times its cost, one per
        hierarchy, up to max_batch."""
        ready = list(self.ready)
        if self.policy == "fifo":  # arrival order, one solve per hierarchy
            batch, seen = [], set()
            for r in ready:
                if len(batch) >= self.max_batch:
                    break
                if r.graph_id not in seen:
                    seen.add(r.graph_id)
                    batch.append(r)
            return batch
        late = [r for r in ready if now - r.t_arrive > self.max_wait_s]
        if late:
            first = min(late, key=lambda r: r.t_arrive)
        else:
            first = min(ready, key=lambda r: (self._req_cost(r), r.t_arrive))
        limit = self.cost_ratio * self._req_cost(first)
        batch, seen = [first], {first.graph_id}
        for r in sorted(ready, key=lambda r: (self._req_cost(r), r.t_arrive)):
            if len(batch) >= self.max_batch:
                break
            if r is first or r.graph_id in seen or self._req_cost(r) > limit:
                continue
            seen.add(r.graph_id)
            batch.append(r)
        return batch

    def _evict_for(self, need: int) -> bool:
        """Free least recently used idle hierarchies until `need` fits."""
        while self.used + self.reserved + need > self.budget:
            victim = None
            for gid, (h, b, users) in self.resident.items():
                if users == 0:
                    victim = gid
                    break
            if victim is None:
                return False
            h, b, _ = self.resident.pop(victim)
            self.backend.free(h)
            self.used -= b
            self.evictions += 1
        return True

    def _admit(self):
        """Admission by footprint, in arrival order (caller holds the lock)."""
        self._drop_stale(time.perf_counter())
        while self.pending:
            req = self.pending[0]
            if req.graph_id in self.resident:
                ent = self.resident[req.graph_id]
                ent[2] += 1
                self.resident.move_to_end(req.graph_id)
                self.pending.popleft()
                req.t_admit = req.t_ready = time.perf_counter()
                req.resident_hit = True
                req.status = "ready"
                self.ready.append(req)
                continue
            need = estimate_footprint(req.n, int(req.col.shape[0]))
            if need > self.budget:
                self.pending.popleft()
                req.status = "rejected"
                req.error = f"footprint {need} exceeds budget {self.budget}"
                req.t_done = time.perf_counter()
                req.event.set()
                self.done.append(req)
                continue
            if not self._evict_for(need):
                break
            self.pending.popleft()
            self.reserved += need
            req._reserved = need
            req.t_admit = time.perf_counter()
            req.status = "admitted"
            self.setup_q.append(req)
        self.peak = max(self.peak, self.used + self.reserved)

    def _setup_loop(self):
        while True:
            with self.lock:
                while not self.setup_q and not self.stop:
                    self.lock.wait()
                if self.stop and not self.setup_q:
                    return
                req = self.setup_q.popleft()
                if req.cancelled or req.expired(time.perf_counter()):
                    self.reserved -= req._reserved
                    self._finish(req, "cancelled" if req.cancelled else "timeout")
                    self._admit()
                    self.lock.notify_all()
                    continue
            try:
                h, nbytes = self.backend.setup(req)
                err = None
            except Exception as e:  # a failed setup fails this request only
                h, nbytes, err = None, 0, str(e)
            with self.lock:
                self.reserved -= req._reserved
                if err is not None:
                    req.status = "failed"
                    req.error = err
                    req.t_done = time.perf_counter()
                    req.event.set()
                    self.done.append(req)
                else:
                    if req.graph_id in self.resident:  # built twice concurrently: keep one
                        self.backend.free(h)
                        ent = self.resident[req.graph_id]
                        ent[2] += 1
                    else:
                        self.resident[req.graph_id] = [h, nbytes, 1]
                        self.used += nbytes
                    req.t_ready = time.perf_counter()
                    req.status = "ready"
                    self.ready.append(req)
                self._admit()
                self.lock.notify_all()

    def _solve_loop(self):
        while True:
            with self.lock:
                while not self.ready and not self.stop:
                    self.lock.wait()
                if self.stop and not self.ready and not self.setup_q and not self.pending:
                    return
                self._drop_stale(time.perf_counter())
                if not self.ready:
                    self.lock.wait(0.01)
                    continue
                batch = self._pick_batch(time.perf_counter())
                for req in batch:
                    self.ready.remove(req)
                    req.status = "solving"
                handles = [self.resident[r.graph_id][0] for r in batch]
            t0 = time.perf_counter()
            try:
                lams, xs = self.backend.solve(handles, [r.n for r in batch])
                err = None
            except Exception as e:
                lams, xs, err = [float("nan")] * len(batch), [None] * len(batch), str(e)
            now = time.perf_counter()
            with self.lock:
                self.batches.append(len(batch))
                if err is None and len(batch) == 1:  # a solo solve measures the graph's cost
                    self.cost[batch[0].graph_id] = now - t0
                elif err is None:
                    for r in batch:  # a batch bounds each member's cost from above
                        self.cost.setdefault(r.graph_id, now - t0)
                for req, lam, x in zip(batch, lams, xs):
                    req.lam, req.x = lam, x
                    req.t_done = now
                    req.status = "done" if err is None else "failed"
                    req.error = err or ""
                    ent = self.resident.get(req.graph_id)
                    if ent is not None:
                        ent[2] -= 1
                    req.event.set()
                    self.done.append(req)
                if self.resident_cap is not None:
                    while len(self.resident) > self.resident_cap and self._evict_one():
                        pass
                self._admit()
                self.lock.notify_all()

    def _evict_one(self) -> bool:
        for gid, (h, b, users) in self.resident.items():
            if users == 0:
                self.resident.pop(gid)
                self.backend.free(h)
                self.used -= b
                self.evictions += 1
                return True
        return False


def latency_summary(reqs) -> dict:
    lat = np.array([r.latency for r in reqs if r.status == "done"])
    if lat.size == 0:
        return {"completed": 0}
    small = [r.latency for r in reqs if r.status == "done" and r.n <= 100_000]
    t0 = min(r.t_arrive for r in reqs)
    t1 = max(r.t_done for r in reqs)
    return {
        "completed": int(lat.size),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "solves_per_s": float(lat.size / (t1 - t0)),
        "resident_hit_rate": float(np.mean([r.resident_hit for r in reqs if r.status == "done"])),
        "p99_small_ms": float(np.percentile(small, 99) * 1e3) if small else None,  # graphs <= 100k vertices
    }


def replay(server: Server, stream, qps: float, seed: int = 0, progress=None, every: int = 25):
    """Submit `stream` (list of Request) with Poisson arrivals at `qps`;
    returns the requests after all completed.  Interarrival times are
    -ln(1-U)/qps with U from a seeded generator.  `progress(done, total)`
    is called after every `every` completions."""
    rng = np.random.default_rng(seed)
    gaps = -np.log1p(-rng.random(len(stream))) / qps
    t = time.perf_counter()
    for req, gap in zip(stream, gaps):
        t += gap
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)
        req.t_arrive = t
        server.submit(req)
    for i, req in enumerate(stream):
        req.event.wait()
        if progress is not None and (i + 1) % every == 0:
            progress(i + 1, len(stream))
    return stream
