"""Pins of the oracle's recursive spectral bisection (the partitioning use
of the Fiedler vector, Section 1; repeated solves as in the remark on the
coarsest level)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from paper_1412_0565_amd import graphs as G


@pytest.mark.parametrize("n,depth", [(64, 1), (64, 3), (96, 2), (40, 3)])
def test_rsb_path_gives_contiguous_halves(orc, n, depth):
    # the Fiedler vector of a path is monotone (cos(pi (i+1/2)/n), sign from
    # the coarsest rule: increasing), and every half of a path is a path
    part = orc.rsb(G.path(n), depth)
    expect = np.zeros(n, dtype=int)
    bounds = [(0, n, 0)]
    for _ in range(depth):
        nb = []
        for lo, hi, p in bounds:
            mid = lo + (hi - lo) // 2
            expect[lo:mid] = 2 * p
            expect[mid:hi] = 2 * p + 1
            nb += [(lo, mid, 2 * p), (mid, hi, 2 * p + 1)]
        bounds = nb
    assert np.array_equal(part, expect)


def test_rsb_long_grid_cuts_across_the_long_side(orc):
    # 16 x 64 grid (id = 64 r + c): lambda_2 is the simple mode along c, so
    # the halves are c < 32 and c >= 32, then quarters by c
    # (each sub-solve fixes its own sign, so a split's orientation is the
    # coarsest rule's of that subgraph)
    g = G.grid2d(16, 64)
    c = np.arange(g.n) % 64
    assert np.array_equal(orc.rsb(g, 1), (c >= 32).astype(int))
    part = orc.rsb(g, 2)
    assert np.array_equal(part >> 1, c // 32)
    quarters = {frozenset(np.nonzero(c // 16 == q)[0]) for q in range(4)}
    assert {frozenset(np.nonzero(part == p)[0]) for p in range(4)} == quarters


def test_rsb_barbell_separates_the_cliques(orc):
    k = 12
    u, v = np.triu_indices(k, 1)
    uu = np.concatenate([u, u + k, [k - 1]])
    vv = np.concatenate([v, v + k, [k]])
    g = G.from_edges(2 * k, uu, vv)
    part = orc.rsb(g, 1)
    assert set(part[:k]) == {part[0]} and set(part[k:]) == {1 - part[0]}


def test_components_against_scipy(orc):
    rng = np.random.default_rng(4)
    for n in (50, 400):
        u = rng.integers(0, n, n // 2)
        v = rng.integers(0, n, n // 2)
        keep = u != v
        g = G.from_edges(n, u[keep], v[keep])
        comp = orc.components(g)
        a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(n, n))
        nc, lab = connected_components(a, directed=False)
        assert len(set(comp)) == nc
        for c in range(nc):
            members = np.nonzero(lab == c)[0]
            assert np.all(comp[members] == members.min())


@pytest.mark.parametrize("name", ["rgg", "cl", "grid"])
def test_rsb_part_sizes_are_balanced(orc, name):
    g = {"rgg": lambda: G.rgg(5000, 10.0, seed=3), "cl": lambda: G.chung_lu(4000, 2.1, 16.0, 300.0, seed=4),
         "grid": lambda: G.grid2d(50, 50)}[name]()
    depth = 4
    part = orc.rsb(g, depth)
    assert part.min() >= 0 and part.max() < 2 ** depth
    # every split is floor/ceil: siblings differ by at most one vertex
    for d in range(depth):
        sizes = np.bincount(part >> (depth - d - 1), minlength=2 ** (d + 1))
        assert np.all(np.abs(sizes[0::2] - sizes[1::2]) <= 1), (d, sizes)
