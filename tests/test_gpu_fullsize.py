"""Full-size parity at the two largest configurations, in the launch
configuration bench.py uses (device arrays, torch allocator and stream).
The oracle's full solve (Algorithms 1-3, single-threaded C) runs in a
thread of its own while the GPU solves.

* 3D 256^3 seven-point grid (16.8M vertices, 100M stored entries, FP32
  input values): FP64 solve against the oracle at the FP64 bar (whole
  hierarchy bit-exact, every step count equal, |cos| >= 1 - 1e-10, lambda
  within 1e-9; its levels 2-4 run one launch per PI step), and the mixed
  solve with every step count equal and lambda within 1e-5 of the oracle.
* Chung-Lu, 4M vertices, exponent 2.1, mean degree 16, cap 50k (FP32
  values; merge-path levels): the same two bars.
* The grid's finest level takes the interleaved row-chunk traversal.
* Both: outputs also checked by properties that hold at any size: unit
  norm, orthogonality to the constant vector, lambda equal to the
  edge-form Rayleigh quotient of the returned vector and the residual equal
  to ||L x - lambda x||, both recomputed in FP64 on the host.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from concurrent.futures import ThreadPoolExecutor

from gpu_compare import MIXED_LAM_RTOL, assert_fp64_parity, assert_refinement_equal, say
from paper_1412_0565_amd import graphs as G

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def solve_device(g, precision, with_arrays=True):
    import torch

    from paper_1412_0565_amd import cmg

    dev = [torch.from_numpy(a).cuda() for a in (g.row_ptr, g.col, g.w)]
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    alloc = cmg.torch_allocator()
    opt = cmg.cmg_options_default(precision=precision, allocator=C.pointer(alloc),
                                  stream=C.c_void_p(torch.cuda.current_stream().cuda_stream))
    h = cmg.cmg_setup(g.n, *dev, opt)
    try:
        st = cmg.cmg_stats()
        st.struct_size = C.sizeof(cmg.cmg_stats)
        lam, _ = cmg.cmg_fiedler(h, x, st)
        levels = cmg.cmg_level_info(h)
        arrays = None
        if with_arrays:
            arrays = [cmg.cmg_level_copy(h, j, levels[j].n, int(levels[j].nnz), with_agg=j < len(levels) - 1)
                      for j in range(len(levels))]
    finally:
        cmg.cmg_free(h)
    return lam, x.cpu().numpy(), st, levels, arrays


def edge_rq_and_residual(g, x):
    """FP64 host recomputation: sum over stored entries w (x_i - x_k)^2 / 2
    over ||x||^2, and ||L x - lam x||."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr.astype(np.int64)))
    w = g.w.astype(np.float64)
    d = x[rows] - x[g.col]
    lam = 0.5 * float(np.dot(w, d * d)) / float(np.dot(x, x))
    lx = np.bincount(rows, weights=w * d, minlength=g.n)  # (L x)_i = sum_k w_ik (x_i - x_k)
    return lam, float(np.linalg.norm(lx - lam * x))


def check_output_properties(g, lam, x, st):
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-12
    assert abs(float(x.sum())) <= 1e-9 * np.sqrt(g.n)
    lam_h, res_h = edge_rq_and_residual(g, x)
    say(f"  lambda {lam!r} host RQ {lam_h!r}; residual {st.residual!r} host {res_h!r}")
    assert abs(lam - lam_h) <= 1e-10 * lam_h
    assert abs(st.residual - res_h) <= 1e-6 * res_h + 1e-12 * (1.0 + lam)


def full_size_case(g, name, expect_step):
    from oracle import oracle as O

    say(f"[fullsize] {name} n={g.n} nnz={g.nnz}: oracle in a thread, GPU FP64 then mixed")
    with ThreadPoolExecutor(1) as ex:
        fut = ex.submit(O.cmg, g)
        lam_d, x_d, st_d, levels_d, arrays = solve_device(g, precision=0)
        say(f"  gpu fp64 lambda {lam_d!r} k {[l.k for l in levels_d]} "
            f"step levels {[j for j, l in enumerate(levels_d) if l.step]} "
            f"merge levels {[j for j, l in enumerate(levels_d) if l.variant == 2]}")
        lam_m, x_m, st_m, levels_m, _ = solve_device(g, precision=1, with_arrays=False)
        say(f"  gpu mixed lambda {lam_m!r} k {[l.k for l in levels_m]} "
            f"fp32 levels {[j for j, l in enumerate(levels_m) if l.fp32]}")
        ref = fut.result()
    say(f"  oracle lambda {ref.lam!r} k {[l.k for l in ref.levels]} residual {ref.residual!r}")
    assert_fp64_parity(g, lam_d, x_d, st_d, levels_d, arrays, ref)
    assert float(np.dot(x_d, ref.y)) > 0
    if expect_step:
        assert any(l.step for l in levels_d)
    check_output_properties(g, lam_d, x_d, st_d)
    assert any(l.fp32 for l in levels_m)
    assert_refinement_equal(ref, levels_m)
    assert abs(lam_m - ref.lam) <= MIXED_LAM_RTOL * ref.lam, (lam_m, ref.lam)
    check_output_properties(g, lam_m, x_m, st_m)
    return levels_d


@pytest.fixture(scope="module")
def grid3d256():
    return G.workload("grid3d256")


def test_fullsize_grid3d256(grid3d256):
    g = grid3d256
    levels = full_size_case(g, "grid3d256", expect_step=True)
    assert levels[0].n == 256 ** 3
    # level 0 walks its rows in chunks interleaved over each XCD's
    # workgroups (more than 4096 rows per workgroup); level 1 and the next
    # run one launch per step
    assert levels[0].variant == 1 and not levels[0].step and levels[0].n > 4096 * levels[0].grid
    assert levels[1].step


@pytest.fixture(scope="module")
def chunglu4m():
    return G.workload("chunglu4m")


def test_fullsize_chunglu4m(chunglu4m):
    levels = full_size_case(chunglu4m, "chunglu4m", expect_step=False)
    assert any(l.variant == 2 for l in levels)
