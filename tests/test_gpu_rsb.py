"""GPU: recursive spectral bisection (cmg_bisect) against the oracle's:
the same part of every vertex, balanced splits, the cut weight."""
import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from gpu_compare import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0565_amd import cmg

    cmg.lib()


CASES = {
    "path64": (lambda: G.path(64), 3),
    "grid16x64": (lambda: G.grid2d(16, 64), 2),
    "rgg20k": (lambda: G.rgg(20000, 10.0, seed=5), 4),
    "rgg60k": (lambda: G.rgg(60000, 10.0, seed=6), 3),
    "cl30k": (lambda: G.chung_lu(30000, 2.1, 16.0, 2000.0, seed=7), 3),
    "grid3d_20": (lambda: G.grid3d(20), 2),
}


def _cut(g, part):
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return 0.5 * float(g.w[part[rows] != part[g.col]].sum())


@pytest.mark.parametrize("name", sorted(CASES))
def test_rsb_parity(name):
    from oracle import oracle as O
    from paper_1412_0565_amd import cmg

    make, depth = CASES[name]
    g = make()
    say(f"[rsb] {name} n={g.n} depth={depth}")
    ref = O.rsb(g, depth)
    part, cut = cmg.cmg_bisect(g.n, g.row_ptr, g.col, g.w, depth)
    say(f"  sizes {np.bincount(part, minlength=2 ** depth).tolist()} cut {cut} mismatches {(part != ref).sum()}")
    assert np.array_equal(part, ref)
    assert cut == pytest.approx(_cut(g, ref), rel=1e-12)


def test_rsb_device_arrays_and_sizes():
    import torch

    from paper_1412_0565_amd import cmg

    g = G.rgg(20000, 10.0, seed=9)
    dev = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col, g.w)]
    part = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    _, cut = cmg.cmg_bisect(g.n, *dev, 5, part=part)
    p = part.cpu().numpy()
    for d in range(5):
        sizes = np.bincount(p >> (5 - d - 1), minlength=2 ** (d + 1))
        assert np.all(np.abs(sizes[0::2] - sizes[1::2]) <= 1)
    assert cut == pytest.approx(_cut(g, p), rel=1e-12)
