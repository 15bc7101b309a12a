"""cmg_fiedler_noalloc (setup + solve + free with every device buffer in the
library's static scratch) against cmg_setup + cmg_fiedler on the same
graphs, two calls in a row (the second on a smaller graph), through the
C ABI."""
import ctypes as C

import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from gpu_compare import COS_TOL, LAM_RTOL, cosine, say

pytestmark = pytest.mark.gpu


def _existing(g, stream, alloc):
    from paper_1412_0565_amd import cmg
    import torch

    dev = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col, g.w)]
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    opt = cmg.cmg_options_default(stream=C.c_void_p(stream), allocator=C.pointer(alloc))
    h = cmg.cmg_setup(g.n, *dev, opt)
    try:
        st = cmg.cmg_stats()
        st.struct_size = C.sizeof(cmg.cmg_stats)
        lam, _ = cmg.cmg_fiedler(h, x, st)
        ks = [l.k for l in cmg.cmg_level_info(h)]
    finally:
        cmg.cmg_free(h)
    return lam, x.cpu().numpy(), st, ks


def test_noalloc_matches_setup_and_fiedler():
    import torch

    from paper_1412_0565_amd import cmg

    assert torch.cuda.is_available()
    stream = torch.cuda.current_stream().cuda_stream
    alloc = cmg.torch_allocator()
    for g in (G.rgg(60000, 10.0, seed=6), G.grid2d(90, 80)):  # second call smaller
        say(f"[noalloc] n={g.n} nnz={g.nnz}")
        dev = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col, g.w)]
        x = torch.full((g.n,), float("nan"), dtype=torch.float64, device="cuda")
        st = cmg.cmg_stats()
        st.struct_size = C.sizeof(cmg.cmg_stats)
        before = torch.cuda.memory_allocated()
        lam, status = cmg.cmg_fiedler_noalloc(g.n, *dev, x,
                                              cmg.cmg_options_default(stream=C.c_void_p(stream)), st)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert status == cmg.CMG_OK
        xn = x.cpu().numpy()
        lam_e, x_e, st_e, ks = _existing(g, stream, alloc)
        c = cosine(xn, x_e)
        say(f"  lambda {lam!r} existing {lam_e!r} 1-cos {1 - c:.2e} bitwise {np.array_equal(xn, x_e)}")
        assert c >= 1 - COS_TOL
        assert abs(lam - lam_e) <= LAM_RTOL * lam_e
        assert st.nlevels == len(ks)
        assert abs(st.residual - st_e.residual) <= 1e-6 * st_e.residual


def test_noalloc_rejects_graphs_beyond_the_scratch():
    from paper_1412_0565_amd import cmg

    g = G.grid2d(700, 700)  # 490k vertices, 1.96M entries: over the 64 MiB bound
    x = np.zeros(g.n)
    with pytest.raises(cmg.CmgError) as ei:
        cmg.cmg_fiedler_noalloc(g.n, g.row_ptr, g.col, g.w, x)
    assert ei.value.status == cmg.CMG_E_ARG
    assert "scratch" in str(ei.value)
