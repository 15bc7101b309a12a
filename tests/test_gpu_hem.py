"""GPU: heavy edge matching (HEM) as the coarsening, the comparison the
paper draws in Section 2.1, against the oracle's HEM mode: matched pairs and
single vertices bit-exact on every level, coarse graphs bit-exact, then the
same refinement bar as HEC."""
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
    "path1000": lambda: G.path(1000),
    "grid128": lambda: G.grid2d(128, 128),
    "grid_aniso": lambda: G.grid2d(90, 77, wx=2.0, wy=1.0),
    "grid3d_20": lambda: G.grid3d(20),
    "rgg60k": lambda: G.rgg(60000, 10.0, seed=6),
    "cl30k": lambda: G.chung_lu(30000, 2.1, 16.0, 2000.0, seed=7),
    "er500": lambda: G.erdos_renyi_connected(500, 0.02, seed=9),
    "star200": lambda: G.star(200),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_hem_parity(name):
    g = GRAPHS[name]()
    say(f"[hem] {name} n={g.n} nnz={g.nnz}")
    ref = oracle_of(g, coarsen=1)
    lam, x, st, levels, arrays = run_gpu(g, coarsen=1)
    say(f"  levels {len(levels)} sizes {[l.n for l in levels][:6]}... k {[l.k for l in levels][-4:]}")
    for a, b in zip(levels, levels[1:]):
        assert 2 * b.n >= a.n  # at most two vertices per aggregate
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("name", ["grid128", "rgg60k"])
def test_hem_mixed(name):
    g = GRAPHS[name]()
    ref = oracle_of(g, coarsen=1)
    lam, x, st, levels, _ = run_gpu(g, want_levels=False, coarsen=1, precision=1, mixed_min_nnz=1)
    assert any(l.fp32 for l in levels)
    assert abs(lam - ref.lam) <= MIXED_LAM_RTOL * ref.lam


def test_hem_and_hec_differ_as_the_lemmas_say():
    # HEC: n_{j+1} <= n_j/2; HEM: n_{j+1} >= n_j/2; both reach the coarsest
    g = G.rgg(60000, 10.0, seed=6)
    _, _, _, hec, _ = run_gpu(g, want_levels=False)
    _, _, _, hem, _ = run_gpu(g, want_levels=False, coarsen=1)
    assert all(2 * b.n <= a.n for a, b in zip(hec, hec[1:]))
    assert all(2 * b.n >= a.n for a, b in zip(hem, hem[1:]))
    assert len(hem) > len(hec)
