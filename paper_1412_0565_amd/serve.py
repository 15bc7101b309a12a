"""Continuous-batching Fiedler server on one GPU.

Requests (a graph and its id) arrive at any time.  The server

* admits a request when its device-memory footprint fits the budget next to
  everything already resident or in flight (admission by HBM footprint);
* builds its hierarchy (``cmg_setup``) on a setup worker with its own HIP
  stream, overlapping the solves of earlier requests;
* solves every request whose hierarchy is ready in the next packed batch
  (``cmg_fiedler_batch``), so requests that arrive while a batch is on the
  GPU join the following one (continuous batching, not a queue);
* keeps hierarchies resident, keyed by graph id, and evicts the least
  recently used ones that are not in use when memory is needed, so a repeat
  graph skips the setup phase;
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
    event: threading.Event = dataclasses.field(default_factory=threading.Event)

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


class Server:
    def __init__(self, backend, budget_bytes: int, max_batch: int = 64, resident_cap: int | None = None):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.resident_cap = resident_cap
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
        return True

    def _admit(self):
        """Admission by footprint, in arrival order (caller holds the lock)."""
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
                if not self.ready:
                    self.lock.wait(0.01)
                    continue
                batch = []
                seen = set()
                for req in list(self.ready):
                    if len(batch) >= self.max_batch:
                        break
                    if req.graph_id in seen:  # one solve per hierarchy per batch
                        continue
                    seen.add(req.graph_id)
                    batch.append(req)
                for req in batch:
                    self.ready.remove(req)
                    req.status = "solving"
                handles = [self.resident[r.graph_id][0] for r in batch]
            try:
                lams, xs = self.backend.solve(handles, [r.n for r in batch])
                err = None
            except Exception as e:
                lams, xs, err = [float("nan")] * len(batch), [None] * len(batch), str(e)
            now = time.perf_counter()
            with self.lock:
                self.batches.append(len(batch))
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
                return True
        return False


def latency_summary(reqs) -> dict:
    lat = np.array([r.latency for r in reqs if r.status == "done"])
    if lat.size == 0:
        return {"completed": 0}
    t0 = min(r.t_arrive for r in reqs)
    t1 = max(r.t_done for r in reqs)
    return {
        "completed": int(lat.size),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "solves_per_s": float(lat.size / (t1 - t0)),
        "resident_hit_rate": float(np.mean([r.resident_hit for r in reqs if r.status == "done"])),
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
