"""GPU: several eigenpairs (Remark after Algorithm 4) through
cmg_fiedler_block against the oracle's block variant: every column at the
FP64 bar (|cos| >= 1 - 1e-10, Rayleigh quotient within 1e-9), equal step
counts on every level, orthonormal output."""
import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from gpu_compare import COS_TOL, LAM_RTOL, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0565_amd import cmg

    cmg.lib()


GRAPHS = {
    "grid60x40": lambda: G.grid2d(60, 40),
    "rgg20k": lambda: G.rgg(20000, 10.0, seed=5),
    "grid3d_20": lambda: G.grid3d(20),
    "cl30k": lambda: G.chung_lu(30000, 2.1, 16.0, 2000.0, seed=7),
    "path1000": lambda: G.path(1000),
}


def _check(g, p, lams, X, res, steps, ref):
    say(f"  lams {lams} oracle {ref.lams}; steps {steps} oracle {ref.k}")
    assert steps == ref.k
    for c in range(p):
        cos = float(X[:, c] @ ref.X[:, c]) / (np.linalg.norm(X[:, c]) * np.linalg.norm(ref.X[:, c]))
        assert cos >= 1 - COS_TOL, (c, cos)
        assert abs(lams[c] - ref.lams[c]) <= LAM_RTOL * ref.lams[c], (c, lams[c], ref.lams[c])
        assert abs(res[c] - ref.residuals[c]) <= 1e-6 * ref.residuals[c] + 1e-12
    assert np.allclose(X.T @ X, np.eye(p), atol=1e-11)
    assert np.allclose(X.sum(0), 0.0, atol=1e-9)


@pytest.mark.parametrize("p", [1, 2, 4])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_block_parity(name, p):
    from oracle import oracle as O
    from paper_1412_0565_amd import cmg

    g = GRAPHS[name]()
    say(f"[block] {name} n={g.n} p={p}")
    ref = O.cmg_block(g, p)
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
        if ref.status == "E_ARG":  # the coarsest level is too small for p columns (or not dense)
            with pytest.raises(cmg.CmgError) as ei:
                F.solve_block(p)
            assert ei.value.status == cmg.CMG_E_ARG
            say(f"  coarsest level {F.levels()[-1].n} vertices: p={p} rejected on both sides")
            return
        lams, X, res, steps = F.solve_block(p)
    assert ref.status == "OK"
    _check(g, p, lams, X, res, steps, ref)


@pytest.mark.parametrize("name", ["grid60x40", "rgg20k"])
def test_block_fixed_schedule(name):
    from oracle import oracle as O
    from paper_1412_0565_amd import cmg

    g = GRAPHS[name]()
    ref = O.cmg_block(g, 3, fixed_k0=3, fixed_beta=1.6)
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w, fixed_k0=3, fixed_beta=1.6) as F:
        lams, X, res, steps = F.solve_block(3)
    _check(g, 3, lams, X, res, steps, ref)


def test_block_reuses_the_hierarchy_and_repeats():
    from paper_1412_0565_amd import cmg

    g = GRAPHS["rgg20k"]()
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
        a = F.solve_block(2)
        lam, x, _ = F.solve()            # the single-vector solve on the same handle
        b = F.solve_block(2)
        c = F.solve_block(3)             # another block width reallocates
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])
    assert abs(float(x @ a[1][:, 0])) > 0.9  # first column near the Fiedler vector
    assert c[0].shape == (3,)


def test_block_rejects_p_beyond_the_coarsest():
    from paper_1412_0565_amd import cmg

    g = G.path(20)  # dense-only: 20 vertices
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
        for p in (20, 5):  # p must stay below the coarsest size and at most 4
            with pytest.raises(cmg.CmgError) as ei:
                cmg.cmg_fiedler_block(F.handle, p)
            assert ei.value.status == cmg.CMG_E_ARG
