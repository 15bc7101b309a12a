"""Generators: exact sizes, symmetry, determinism (CPU)."""
import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G


def _check_csr(g):
    rp, col, w = g.row_ptr, g.col, g.w
    assert rp.dtype == np.int32 and col.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == col.size == w.size
    assert np.all(np.diff(rp) >= 1), "isolated vertex"
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col != rows), "self loop"
    assert np.all((col >= 0) & (col < g.n))
    for i in range(min(g.n, 2000)):
        seg = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)
    assert np.all(w > 0)
    # symmetry: (i, k, w) present iff (k, i, w) present
    key1 = rows.astype(np.int64) * g.n + col
    key2 = col.astype(np.int64) * g.n + rows
    o1 = np.argsort(key1)
    o2 = np.argsort(key2)
    assert np.array_equal(key1[o1], key2[o2])
    assert np.array_equal(w[o1], w[o2])


def test_grid2d_sizes():
    g = G.grid2d(128, 128)
    assert g.n == 16384 and g.m == 2 * 128 * 127 and g.nnz == 65024
    _check_csr(g)


@pytest.mark.parametrize("s", [2, 3, 7, 16])
def test_grid3d_sizes(s):
    g = G.grid3d(s)
    assert g.n == s ** 3 and g.m == 3 * s * s * (s - 1)
    _check_csr(g)
    # same graph through the generic edge-list builder
    idx = np.arange(g.n).reshape(s, s, s)  # [z, y, x]
    u = np.concatenate([idx[:, :, :-1].ravel(), idx[:, :-1, :].ravel(), idx[:-1].ravel()])
    v = np.concatenate([idx[:, :, 1:].ravel(), idx[:, 1:, :].ravel(), idx[1:].ravel()])
    h = G.from_edges(g.n, u, v)
    assert np.array_equal(h.row_ptr, g.row_ptr) and np.array_equal(h.col, g.col)


def test_closed_families():
    for g, m in [(G.path(10), 9), (G.cycle(10), 10), (G.complete(7), 21), (G.star(9), 8)]:
        _check_csr(g)
        assert g.m == m


def test_rgg_small_deterministic():
    a = G.rgg(20000, 10.0, seed=7)
    b = G.rgg(20000, 10.0, seed=7)
    c = G.rgg(20000, 10.0, seed=8)
    _check_csr(a)
    assert G.is_connected(a)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w)
    assert not (a.n == c.n and np.array_equal(a.col[:100], c.col[:100]))
    assert set(np.unique(a.w)) <= set(range(1, 9))
    assert 8.5 < a.nnz / a.n < 11.0


def test_chung_lu_small():
    g = G.chung_lu(50000, 2.1, 16.0, 2000.0, seed=3)
    _check_csr(g)
    assert G.is_connected(g)
    deg = np.diff(g.row_ptr)
    assert deg.max() > 20 * np.median(deg)  # skewed


def test_chung_lu_weights_mean():
    w = G.chung_lu_weights(4_000_000, 2.1, 16.0, 50000.0)
    assert abs(w.mean() - 16.0) < 1e-9
    assert (w >= 50000.0 - 1e-6).sum() >= 10


def test_stream_is_splitmix64():
    # i-th output of stream (seed, tag) == SplitMix64 sequence started at state0
    s0 = int(G._state0(5, 9))
    M = (1 << 64) - 1
    exp = []
    st = s0
    for _ in range(4):
        st = (st + 0x9E3779B97F4A7C15) & M
        z = st
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        exp.append(z ^ (z >> 31))
    got = G.stream_u64(5, 9, np.arange(4, dtype=np.uint64))
    assert [int(x) for x in got] == exp
