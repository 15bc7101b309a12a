"""Pins of the oracle's two variations (CPU): Algorithm 4's fixed smoothing
schedule k_j = beta^j k_0 (Section 3, main theorem and the complexity
corollary), and heavy edge matching (HEM) as the coarsening of Step 1
(Section 2.1, the lemma on coarsening rates)."""
import itertools
import math

import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from test_oracle import _path_modes, _small_graphs


# ------------------------------------------------------------ fixed schedule

@pytest.mark.parametrize("k0,beta,expect", [
    (1, 2.0, [1, 2, 4, 8, 16, 32]),
    (2, 1.5, [2, 3, 5, 7, 11, 16]),     # 2 * 1.5^j = 2, 3, 4.5, 6.75, 10.125, 15.1875
    (3, 1.0, [3, 3, 3, 3, 3, 3]),
    (1, 4.0, [1, 4, 16, 64, 256, 1024]),  # beta = 4, k_0 = 1: the paper's Table 4 setting
])
def test_fixed_steps_schedule(orc, k0, beta, expect):
    assert [orc.fixed_steps(k0, beta, j) for j in range(6)] == expect


def test_fixed_steps_cap(orc):
    assert orc.fixed_steps(5, 10.0, 9, 1000) == 1000
    assert orc.fixed_steps(5, 10.0, 2, 1000) == 500


def test_pi_fixed_exact_eigenvector_stays(orc):
    # B_g maps an eigenvector phi_2 (orthogonal to 1) onto (g - lambda_2) phi_2,
    # so every fixed step returns the same unit vector
    n = 30
    g = G.path(n)
    modes, lam = _path_modes(n)
    for steps in (1, 7, 40):
        y, utv = orc.pi_fixed(g, modes[1], steps)
        assert np.allclose(y, modes[1], atol=1e-13)
        assert abs(utv - 1.0) < 1e-13


def test_pi_fixed_rate_is_the_power_iteration_ratio(orc):
    # u^0 = phi_2 + eps phi_3 on a path (closed-form modes): after k steps of
    # B_g = gI - L the phi_3/phi_2 coefficient ratio is eps ((g-l3)/(g-l2))^k
    # exactly (power-iteration theorem of Section 2.2); no stopping test.
    n = 24
    g = G.path(n)
    modes, lam = _path_modes(n)
    gv = orc.gershgorin(g)
    eps = 0.25
    u0 = modes[1] + eps * modes[2]
    r = (gv - lam[2]) / (gv - lam[1])
    for k in (1, 3, 10, 50):
        y, _ = orc.pi_fixed(g, u0, k)
        c2, c3 = y @ modes[1], y @ modes[2]
        assert c3 / c2 == pytest.approx(eps * r ** k, rel=1e-10)
        assert abs(y.sum()) < 1e-13 and abs(np.linalg.norm(y) - 1) < 1e-14


def test_pi_fixed_equals_pi_without_test(orc):
    # the tolerance-mode iteration with the test disabled (tol < 0) and the
    # cap at k performs the same k steps in the same order
    g = G.rgg(3000, 10.0, seed=3)
    y0 = np.array([orc.uniform(7, i) for i in range(g.n)]) - 0.5
    a, _ = orc.pi_fixed(g, y0, 17)
    b, k, _ = orc.pi(g, y0, tol=-1.0, maxit=17)
    assert k == 17 and np.array_equal(a, b)


def test_cmg_fixed_schedule_step_counts(orc):
    g = G.grid2d(100, 100)
    r = orc.cmg(g, fixed_k0=3, fixed_beta=1.6)
    assert r.status == "OK"
    J = len(r.levels) - 1
    assert [lv.k for lv in r.levels[:J]] == [orc.fixed_steps(3, 1.6, j) for j in range(J)]
    assert r.levels[J].k == -1
    # same hierarchy as the tolerance mode: only Step 3 changes
    t = orc.cmg(g)
    assert [lv.n for lv in r.levels] == [lv.n for lv in t.levels]
    lam2 = 2 - 2 * math.cos(math.pi / 100)
    assert r.lam >= lam2 * (1 - 1e-12)
    assert abs(r.y.sum()) < 1e-10 and abs(np.linalg.norm(r.y) - 1) < 1e-13


def test_cmg_fixed_schedule_error_falls_with_k0(orc):
    # main theorem: the eigenvector error is bounded by C h_0^a / k_0^(a/2)
    # (beta > 4); the eigenvalue error r - lambda_2 falls as k_0 grows
    g = G.grid2d(128, 128)
    lam2 = 2 - 2 * math.cos(math.pi / 128)
    errs = [orc.cmg(g, fixed_k0=k0, fixed_beta=4.5).lam - lam2 for k0 in (1, 4, 16)]
    assert errs[0] > errs[1] > errs[2] > 0


def test_cmg_fixed_dense_only_is_exact(orc):
    g = G.path(20)  # n <= 25: the coarsest level is the graph, no smoothing
    r = orc.cmg(g, fixed_k0=2, fixed_beta=2.0)
    assert len(r.levels) == 1 and r.levels[0].k == -1
    assert r.lam == pytest.approx(2 - 2 * math.cos(math.pi / 20), rel=1e-13)


# ----------------------------------------------------------------------- HEM

def _hem_by_edge_order(g, order):
    """Independent formulation: HEM is the greedy maximal matching that
    takes the edges in the order (rank of the endpoint visited first,
    decreasing weight, index of the other endpoint), accepting an edge when
    both endpoints are free.  (When a vertex's turn comes every earlier
    neighbour is already matched, so its unmatched neighbours are later
    ones; the heaviest of them is its first free edge in this order.)
    Single vertices open their own aggregate; ids by ascending opener."""
    n = g.n
    rank = np.empty(n, dtype=np.int64)
    rank[np.asarray(order)] = np.arange(n)
    edges = []
    for a in range(n):
        for e in range(g.row_ptr[a], g.row_ptr[a + 1]):
            b = int(g.col[e])
            if rank[a] < rank[b]:
                edges.append((rank[a], -g.w[e], b, a))
    edges.sort()
    opener = np.full(n, -1)
    for _, _, b, a in edges:
        if opener[a] < 0 and opener[b] < 0:
            opener[a] = opener[b] = a
    for v in range(n):
        if opener[v] < 0:
            opener[v] = v
    seeds = sorted(set(int(o) for o in opener))
    idx = {s: i for i, s in enumerate(seeds)}
    return np.array([idx[int(o)] for o in opener]), len(seeds)


def _hem_by_rounds(g, key):
    """Round-synchronous formulation the GPU kernels use: in each round a
    live vertex whose live neighbours all come later in the key order
    proposes to its heaviest live neighbour (lowest index on ties); the
    proposal is accepted when the proposer is that neighbour's earliest live
    neighbour; a live vertex with no live neighbour left stays alone."""
    n = g.n
    live = np.ones(n, dtype=bool)
    opener = np.full(n, -1)
    rounds = 0
    while live.any():
        rounds += 1
        mkey = np.full(n, np.iinfo(np.uint64).max, dtype=np.uint64)
        for v in np.nonzero(live)[0]:
            for e in range(g.row_ptr[v], g.row_ptr[v + 1]):
                u = g.col[e]
                if live[u] and key[u] < mkey[v]:
                    mkey[v] = key[u]
        accept = []
        for v in np.nonzero(live)[0]:
            nb = [(g.w[e], -int(g.col[e])) for e in range(g.row_ptr[v], g.row_ptr[v + 1]) if live[g.col[e]]]
            if not nb:
                accept.append((v, -1))
                continue
            if key[v] > mkey[v]:
                continue
            best = -max(nb)[1]
            if mkey[best] == key[v]:
                accept.append((v, best))
        for v, u in accept:
            opener[v] = v
            live[v] = False
            if u >= 0:
                opener[u] = v
                live[u] = False
    seeds = sorted(set(int(o) for o in opener))
    idx = {s: i for i, s in enumerate(seeds)}
    return np.array([idx[int(o)] for o in opener]), len(seeds), rounds


def test_hem_path6_by_hand(orc):
    g = G.from_edges(6, [0, 1, 2, 3, 4], [1, 2, 3, 4, 5], [3.0, 1.0, 2.0, 5.0, 1.0])
    agg, seed, nc = orc.hem_order(g, [0, 1, 2, 3, 4, 5])
    assert nc == 3 and list(agg) == [0, 0, 1, 1, 2, 2]
    # 3 takes its heaviest free neighbour 4 (weight 5); 0 takes 1; 2 and 5 are left alone
    agg, seed, nc = orc.hem_order(g, [3, 0, 1, 2, 4, 5])
    assert nc == 4 and list(agg) == [0, 0, 1, 2, 2, 3]
    assert list(np.nonzero(seed)[0]) == [0, 2, 3, 5]


def test_hem_ties_lowest_index(orc):
    g = G.from_edges(4, [0, 0, 0], [1, 2, 3], [2.0, 5.0, 5.0])
    agg, _, nc = orc.hem_order(g, [0, 1, 2, 3])
    assert nc == 3 and agg[0] == agg[2] and len({agg[1], agg[3], agg[0]}) == 3


def test_hem_all_visit_orders_match_edge_order_formulation(orc):
    total = 0
    for g in _small_graphs():
        for order in itertools.permutations(range(g.n)):
            agg, _, nc = orc.hem_order(g, list(order))
            agg2, nc2 = _hem_by_edge_order(g, order)
            assert nc == nc2 and np.array_equal(agg, agg2), (g.n, order)
            total += 1
    assert total > 20000


def test_hem_rounds_formulation_matches_oracle(orc):
    for name, g in [("rgg", G.rgg(3000, 10.0, seed=11)), ("grid", G.grid2d(30, 40)),
                    ("cl", G.chung_lu(3000, 2.1, 16.0, 300.0, seed=2))]:
        for level in (0, 3):
            agg, _, nc = orc.hem(g, 14120565, level)
            key = np.array([orc.hec_key(14120565, level, v) for v in range(g.n)], dtype=np.uint64)
            agg2, nc2, rounds = _hem_by_rounds(g, key)
            assert nc == nc2 and np.array_equal(agg, agg2), name
            assert rounds < 60


@pytest.mark.parametrize("gname", ["rgg", "grid", "cl"])
def test_hem_invariants(orc, gname):
    g = {"rgg": lambda: G.rgg(5000, 10.0, seed=4), "grid": lambda: G.grid2d(50, 60),
         "cl": lambda: G.chung_lu(5000, 2.1, 16.0, 500.0, seed=5)}[gname]()
    agg, seed, nc = orc.hem(g, 14120565, 0)
    sizes = np.bincount(agg, minlength=nc)
    assert sizes.min() >= 1 and sizes.max() <= 2
    assert nc >= (g.n + 1) // 2          # lemma on coarsening rates: k_M >= 1/2
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    # pairs are edges
    for a in np.nonzero(sizes == 2)[0][:2000]:
        u, v = np.nonzero(agg == a)[0]
        assert v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]
    # maximal: no edge joins two single vertices
    single = sizes[agg] == 1
    assert not np.any(single[rows] & single[g.col])


def test_hem_hierarchy_is_deeper_than_hec(orc):
    # HEC aggregates have two vertices or more (n_{j+1} <= n_j/2); HEM's
    # have at most two (n_{j+1} >= n_j/2)
    g = G.grid2d(100, 100)
    a = orc.cmg(g)
    b = orc.cmg(g, coarsen="hem")
    assert len(b.levels) > len(a.levels)
    for x, y in zip(b.levels, b.levels[1:]):
        assert 2 * y.n >= x.n
    lam2 = 2 - 2 * math.cos(math.pi / 100)
    assert b.lam >= lam2 * (1 - 1e-12)
    assert abs(b.y.sum()) < 1e-10 and abs(np.linalg.norm(b.y) - 1) < 1e-13


def test_cmg_hem_vs_dense_eigensolver(orc):
    g = G.rgg(2000, 10.0, seed=21)
    a = g.to_dense()
    ev = np.linalg.eigvalsh(np.diag(a.sum(1)) - a)
    r = orc.cmg(g, coarsen="hem", tol=1e-15, max_iters=200000)
    assert abs(r.lam - ev[1]) < 1e-5 * ev[1]
