"""Continuous-batching server on the GPU: requests of different sizes and
precisions arrive while others are being solved; every result must equal
the solo solve of the same graph bit for bit (same kernels, same workgroup
counts), and the server must actually batch."""
import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from gpu_compare import say

pytestmark = pytest.mark.gpu


def _pool():
    return [("rgg5k", G.rgg(5000, 10.0, seed=31), 0),
            ("rgg40k", G.rgg(40000, 10.0, seed=32), 0),
            ("rgg40k_mixed", G.rgg(40000, 10.0, seed=32), 1),
            ("grid60", G.grid2d(60, 60), 0),
            ("cl20k", G.chung_lu(20000, 2.5, 8.0, 400.0, seed=33, int_weights=True), 0),
            ("grid3d_24", G.grid3d(24), 1)]


def test_served_results_equal_solo():
    import torch
    from paper_1412_0565_amd import cmg
    from paper_1412_0565_amd.serve import CmgBackend, Request, Server, latency_summary, replay

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pool = _pool()
    solo = {}
    for name, g, prec in pool:
        with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w, precision=prec) as F:
            lam, x, _ = F.solve()
        solo[name] = (lam, x)
        say(f"[serve] solo {name} lambda={lam:.10e}")
    backend = CmgBackend()
    srv = Server(backend, budget_bytes=2 << 30, max_batch=8, resident_cap=3)
    try:
        stream = []
        for i in range(30):
            name, g, prec = pool[(i * 7) % len(pool)]
            stream.append(Request(i, name, g.n, g.row_ptr, g.col, g.w, precision=prec))
        replay(srv, stream, qps=2000.0, seed=4)
        # graphs still resident after the stream are served from their kept
        # hierarchies (whether the stream itself hit depends on timing)
        with srv.lock:
            kept = list(srv.resident.keys())
        assert kept
        by_name = {name: (g, prec) for name, g, prec in pool}
        again = []
        for i, name in enumerate(kept):
            g, prec = by_name[name]
            again.append(Request(1000 + i, name, g.n, g.row_ptr, g.col, g.w, precision=prec))
        replay(srv, again, qps=2000.0, seed=5)
    finally:
        srv.close()
    assert all(r.resident_hit for r in again)
    stream = stream + again
    for r in stream:
        assert r.status == "done", (r.rid, r.status, r.error)
        lam, x = solo[r.graph_id]
        assert r.lam == lam, (r.graph_id, r.lam, lam)
        assert np.array_equal(r.x, x), r.graph_id
    say(f"[serve] batches {srv.batches} summary {latency_summary(stream)}")
    assert max(srv.batches) >= 2
