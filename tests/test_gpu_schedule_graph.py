"""GPU: the fixed smoothing schedule (Algorithm 4's k_j = beta^j k_0 on the
algebraic hierarchy) against the oracle's fixed mode, and HIP-graph replay
of a solve's launch sequence against eager launches."""
import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from gpu_compare import MIXED_LAM_RTOL, assert_fp64_parity, oracle_of, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0565_amd import cmg

    cmg.lib()


GRAPHS = {
    "grid128": lambda: G.grid2d(128, 128),
    "rgg60k": lambda: G.rgg(60000, 10.0, seed=6),
    "cl30k": lambda: G.chung_lu(30000, 2.1, 16.0, 2000.0, seed=7),
    "grid3d_20": lambda: G.grid3d(20),
    "star200": lambda: G.star(200),
    "path1000": lambda: G.path(1000),
}


def _schedule(k0, beta, j):
    from oracle import oracle as O

    return O.fixed_steps(k0, beta, j)


@pytest.mark.parametrize("graph", [0, 1])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_fixed_schedule_parity(name, graph):
    from paper_1412_0565_amd import cmg

    g = GRAPHS[name]()
    opts = dict(fixed_k0=3, fixed_beta=1.6)
    say(f"[fixed] {name} n={g.n} graph={graph}")
    ref = oracle_of(g, **opts)
    lam, x, st, levels, arrays = run_gpu(g, graph=graph, **opts)
    say(f"  k {[l.k for l in levels]} oracle {[l.k for l in ref.levels]}")
    assert st.status == cmg.CMG_OK
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)
    for j, lv in enumerate(levels):
        if lv.k != -1:
            assert lv.k == _schedule(3, 1.6, j)


@pytest.mark.parametrize("name", ["grid128", "rgg60k", "grid3d_20"])
def test_fixed_schedule_step_mode_in_graph(name):
    # every grid level one launch per step with a known count: the whole
    # refinement, step launches included, is one captured graph
    g = GRAPHS[name]()
    opts = dict(fixed_k0=2, fixed_beta=2.0)
    ref = oracle_of(g, **opts)
    lam, x, st, levels, arrays = run_gpu(g, graph=1, step_mode=1, block_rows=1, **opts)
    assert any(l.step for l in levels)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("name", ["grid128", "rgg60k"])
def test_fixed_schedule_mixed(name):
    g = GRAPHS[name]()
    opts = dict(fixed_k0=3, fixed_beta=1.6)
    ref = oracle_of(g, **opts)
    lam, x, st, levels, _ = run_gpu(g, want_levels=False, graph=1, precision=1, mixed_min_nnz=1, **opts)
    assert any(l.fp32 for l in levels)
    assert abs(lam - ref.lam) <= MIXED_LAM_RTOL * ref.lam, (lam, ref.lam)
    assert [l.k for l in levels] == [l.k for l in ref.levels]


def _solve_many(h, n, reps, between):
    from paper_1412_0565_amd import cmg

    out = []
    for r in range(reps):
        x = np.zeros(n)
        lam, _ = cmg.cmg_fiedler(h, x)
        out.append((lam, x))
        between(r)
    return out


@pytest.mark.parametrize("opts", [dict(), dict(fixed_k0=3, fixed_beta=1.6), dict(precision=1, mixed_min_nnz=1)])
def test_graph_replays_equal_eager(opts):
    """Graph replays, with other eager work and synchronisations between
    them, give bitwise the result of eager launches, every time."""
    import torch

    from paper_1412_0565_amd import cmg

    g = G.rgg(60000, 10.0, seed=6)
    other = G.grid2d(90, 80)
    say(f"[graph] rgg60k {opts}")
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w, graph=0, **opts) as E:
        lam_e, x_e, _ = E.solve()
        assert not any(l.step for l in E.levels())

    def eager_work(r):
        with cmg.Fiedler(other.n, other.row_ptr, other.col, other.w) as H:
            H.solve()
        t = torch.ones(1 << 20, device="cuda") * (r + 1)
        torch.cuda.synchronize()
        assert float(t.sum()) == float((r + 1) << 20)

    h = cmg.cmg_setup(g.n, g.row_ptr, g.col, g.w, cmg.cmg_options_default(graph=1, **opts))
    try:
        runs = _solve_many(h, g.n, 5, eager_work)
    finally:
        cmg.cmg_free(h)
    for lam, x in runs:
        assert lam == lam_e
        assert np.array_equal(x, x_e)


def test_graph_skipped_when_steps_are_decided_on_the_host():
    # tolerance mode with step-mode levels: the step count of those levels
    # is read back by the host, so the solve runs eagerly (same results)
    g = G.grid3d(128)
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, graph=1)
    assert any(l.step for l in levels)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("name", ["rgg60k", "cl30k", "grid3d_20"])
def test_autotuner_against_oracle_and_repeatable(name):
    """autotune=1 times candidate lanes-per-row and workgroup counts of each
    grid level with real PI steps and keeps the fastest; the solve still
    matches the oracle, and within a process the choice (cached by level
    shape) and so the result repeat bitwise."""
    from paper_1412_0565_amd import cmg

    g = GRAPHS[name]()
    say(f"[autotune] {name}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, autotune=1)
    say(f"  lanes {[l.lanes for l in levels]} grid {[l.grid for l in levels]}")
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)
    lam2, x2, _, levels2, _ = run_gpu(g, want_levels=False, autotune=1)
    assert [(l.lanes, l.grid) for l in levels2] == [(l.lanes, l.grid) for l in levels]
    assert lam2 == lam and np.array_equal(x2, x)
