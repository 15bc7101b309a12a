"""Host-side accounting of bench.py (no GPU): algorithmic bytes of the
level-0 refinement launch and of setup, the counter-file lookup, and the
one-GPU guard."""
from __future__ import annotations

import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def level(n, nnz, k=0, weights=0, fp32=0):
    sx = 4 if fp32 else 8
    sw = {0: 8, 1: 4, 2: 0, 3: 1, 4: 2}[weights]
    return types.SimpleNamespace(n=n, nnz=nnz, k=k, weights=weights, fp32=fp32,
                                 bytes_per_iter=4 * (n + 1) + nnz * (4 + sw) + 2 * sx * n)


def test_level0_launch_bytes_of_the_256_grid():
    # 5 PI steps of 4(n+1) + 4 nnz + 16 n (unit weights, none read) plus
    # the prolongation (aggregate read, coarse gather, write) and the pass
    # over the start vector: 5 * 736,624,644 + 384,865,208
    lv = [level(256 ** 3, 100270080, k=5, weights=2), level(6165111, 52241808, k=18, weights=3)]
    assert lv[0].bytes_per_iter == 736624644
    assert bench.launch_bytes(lv, 0) == 4067988428


def test_setup_bytes_by_hand():
    # one coarsened level: row pass 4(n+1) + 12 nnz, Galerkin read
    # 4(n+1) + 16 nnz + 4 n, coarse CSR 4(nc+1) + 12 nnz_c
    lv = [level(10, 40, weights=0), level(4, 12, weights=0)]
    want = (44 + 480) + (44 + 640 + 40) + (20 + 144)
    assert bench.setup_bytes(lv) == want
    # unit weights are not read
    lv[0].weights = 2
    assert bench.setup_bytes(lv) == want - 8 * 40 * 2
    r = bench.setup_roofline(lv, 1e-3)  # 772 bytes in 1 us: 0.772 GB/s
    assert r["bytes"] == 772 and r["unit"] == "GB/s" and r["achieved"] == pytest.approx(0.8, abs=0.05)


def test_counter_file_lookup_needs_matching_step_count():
    got, src = bench.measured_traffic("grid3d256", types.SimpleNamespace(k=5))
    if got is None:
        pytest.skip(f"counter summary not on these kernel sources: {src}")
    assert got > 4067988428  # measured traffic includes some re-fetch
    stale, src = bench.measured_traffic("grid3d256", types.SimpleNamespace(k=6))
    assert stale is None and "stale" in src
    none, src = bench.measured_traffic("no_such_workload", types.SimpleNamespace(k=5))
    assert none is None and src is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "--gpus 1" in r.stderr
