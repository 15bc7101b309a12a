"""Scheduler logic of the continuous-batching server, driven on the CPU by
a fake backend (no GPU): admission by footprint, batching of requests that
arrive during a solve, residency hits, eviction, failure isolation."""
import threading
import time

import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G
from paper_1412_0565_amd.serve import Request, Server, estimate_footprint, latency_summary, replay


class FakeBackend:
    def __init__(self, setup_s=0.01, solve_s=0.02, fail_ids=()):
        self.setup_s, self.solve_s, self.fail_ids = setup_s, solve_s, set(fail_ids)
        self.lock = threading.Lock()
        self.live = {}
        self.setups = 0
        self.frees = 0
        self.next = 1
        self.batches = []

    def setup(self, req):
        time.sleep(self.setup_s)
        if req.graph_id in self.fail_ids:
            raise RuntimeError("injected setup failure")
        with self.lock:
            h = self.next
            self.next += 1
            self.live[h] = req.graph_id
            self.setups += 1
        return h, estimate_footprint(req.n, int(req.col.shape[0])) // 2

    def solve(self, handles, ns):
        time.sleep(self.solve_s)
        with self.lock:
            self.batches.append(list(handles))
            gids = [self.live[h] for h in handles]
        return [float(hash(g) % 1000) for g in gids], [np.full(n, float(hash(g) % 7)) for g, n in zip(gids, ns)]

    def free(self, h):
        with self.lock:
            del self.live[h]
            self.frees += 1


def _req(rid, gid, n=2000):
    g = G.path(n)
    return Request(rid, gid, g.n, g.row_ptr, g.col, g.w)


def test_requests_during_a_solve_join_the_next_batch():
    be = FakeBackend(setup_s=0.001, solve_s=0.05)
    srv = Server(be, budget_bytes=1 << 30)
    try:
        reqs = [srv.submit(_req(i, f"g{i}")) for i in range(3)]
        time.sleep(0.02)
        later = [srv.submit(_req(10 + i, f"h{i}")) for i in range(5)]
        for r in reqs + later:
            assert r.event.wait(5)
        assert all(r.status == "done" for r in reqs + later)
        assert max(len(b) for b in be.batches) >= 2  # continuous batching, not one at a time
    finally:
        srv.close()


def test_admission_never_exceeds_budget():
    be = FakeBackend(setup_s=0.005, solve_s=0.005)
    one = estimate_footprint(2000, 3998)
    srv = Server(be, budget_bytes=int(2.5 * one))
    try:
        reqs = [srv.submit(_req(i, f"g{i}")) for i in range(12)]
        for r in reqs:
            assert r.event.wait(10)
        assert all(r.status == "done" for r in reqs)
        assert srv.peak <= srv.budget
    finally:
        srv.close()


def test_oversized_request_rejected_others_served():
    be = FakeBackend()
    small = estimate_footprint(2000, 3998)
    srv = Server(be, budget_bytes=int(1.5 * small))
    try:
        big = srv.submit(_req(0, "big", n=50000))
        ok = srv.submit(_req(1, "ok"))
        assert big.event.wait(5) and ok.event.wait(5)
        assert big.status == "rejected" and ok.status == "done"
    finally:
        srv.close()


def test_failed_setup_isolated():
    be = FakeBackend(fail_ids={"bad"})
    srv = Server(be, budget_bytes=1 << 30)
    try:
        rs = [srv.submit(_req(0, "a")), srv.submit(_req(1, "bad")), srv.submit(_req(2, "b"))]
        for r in rs:
            assert r.event.wait(5)
        assert [r.status for r in rs] == ["done", "failed", "done"]
        assert "injected" in rs[1].error
    finally:
        srv.close()


def test_resident_hierarchies_skip_setup_and_evict_lru():
    be = FakeBackend(setup_s=0.001, solve_s=0.001)
    srv = Server(be, budget_bytes=1 << 30, resident_cap=2)
    try:
        for rid, gid in enumerate(["a", "b", "a", "a", "b", "c", "a"]):
            r = srv.submit(_req(rid, gid))
            assert r.event.wait(5)
        done = srv.done
        # after c arrives the cap of 2 evicts the least recently used idle
        # hierarchy (a: last used before b), so the final a is built again
        assert [r.resident_hit for r in done] == [False, False, True, True, True, False, False]
        assert be.setups == 4
        assert len(srv.resident) <= 2
    finally:
        srv.close()
    assert not be.live  # everything freed at close


def test_replay_poisson_and_summary():
    be = FakeBackend(setup_s=0.001, solve_s=0.002)
    srv = Server(be, budget_bytes=1 << 30)
    try:
        stream = [_req(i, f"g{i % 5}") for i in range(40)]
        replay(srv, stream, qps=400.0, seed=1)
    finally:
        srv.close()
    s = latency_summary(stream)
    assert s["completed"] == 40 and s["p99_ms"] >= s["p50_ms"] > 0
    assert 0.5 < s["resident_hit_rate"] <= 1.0


def test_cancel_and_timeout_drop_requests_before_their_batch():
    be = FakeBackend(setup_s=0.001, solve_s=0.2)
    srv = Server(be, budget_bytes=1 << 30, max_batch=1)
    try:
        first = srv.submit(_req(0, "busy"))           # occupies the GPU for 0.2 s
        time.sleep(0.05)
        gone = srv.submit(_req(1, "gone"))
        late = _req(2, "late")
        late.timeout_s = 0.05
        srv.submit(late)
        kept = srv.submit(_req(3, "kept"))
        srv.cancel(gone)
        for r in (first, gone, late, kept):
            assert r.event.wait(5)
    finally:
        srv.close()
    assert first.status == "done" and kept.status == "done"
    assert gone.status == "cancelled" and late.status == "timeout"
    assert be.live == {} or all(v in ("busy", "kept") for v in be.live.values())


def test_batches_group_requests_of_similar_cost():
    be = FakeBackend(setup_s=0.001, solve_s=0.05)
    srv = Server(be, budget_bytes=1 << 30, max_batch=8, cost_ratio=2.0, max_wait_s=10.0)
    try:
        # measured costs: two cheap graphs and one expensive one
        srv.cost.update({"cheap1": 0.001, "cheap2": 0.0015, "dear": 0.2})
        blocker = srv.submit(_req(0, "blocker"))
        time.sleep(0.01)
        reqs = [srv.submit(_req(i + 1, g)) for i, g in enumerate(["dear", "cheap1", "cheap2"])]
        for r in [blocker] + reqs:
            assert r.event.wait(5)
    finally:
        srv.close()
    # the cheap pair shared a batch and it ran before the expensive one
    cheap = [r for r in reqs if r.graph_id.startswith("cheap")]
    dear = [r for r in reqs if r.graph_id == "dear"][0]
    assert cheap[0].t_done == cheap[1].t_done
    assert cheap[0].t_done < dear.t_done
    assert 2 in srv.batches


def test_long_waiting_request_is_not_starved():
    be = FakeBackend(setup_s=0.001, solve_s=0.02)
    srv = Server(be, budget_bytes=1 << 30, max_batch=1, max_wait_s=0.05)
    try:
        srv.cost["dear"] = 1.0
        dear = srv.submit(_req(0, "dear"))
        cheap = []
        for i in range(20):  # a steady supply of cheaper work
            srv.cost[f"c{i}"] = 0.001
            cheap.append(srv.submit(_req(i + 1, f"c{i}")))
            time.sleep(0.01)
        for r in [dear] + cheap:
            assert r.event.wait(5)
    finally:
        srv.close()
    assert dear.t_done < cheap[-1].t_done
