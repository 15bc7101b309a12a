"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Bar: aggregates, coarse CSR and PI step counts bit-exact; FP64 vector
|cos| >= 1 - 1e-10 and eigenvalue relative error <= 1e-9; mixed path
eigenvalue relative error <= 1e-5 against the FP64 oracle.
"""
import math

import numpy as np
import pytest

from paper_1412_0565_amd import graphs as G

from gpu_compare import (MIXED_LAM_RTOL, assert_fp64_parity, cosine, oracle_of, run_gpu, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_0565_amd import cmg

    cmg.lib()


def _named(name):
    return {
        "path2": lambda: G.path(2),
        "path20": lambda: G.path(20),
        "path1000": lambda: G.path(1000),
        "cycle101": lambda: G.cycle(101),
        "K25": lambda: G.complete(25),
        "K60": lambda: G.complete(60),
        "star200": lambda: G.star(200),
        "grid5": lambda: G.grid2d(5, 5),
        "grid100": lambda: G.grid2d(100, 100),
        "grid128": lambda: G.grid2d(128, 128),
        "grid_aniso": lambda: G.grid2d(90, 77, wx=2.0, wy=1.0),
        "grid3d_20": lambda: G.grid3d(20),
        "rgg20k": lambda: G.rgg(20000, 10.0, seed=5),
        "rgg60k": lambda: G.rgg(60000, 10.0, seed=6),
        "cl30k": lambda: G.chung_lu(30000, 2.1, 16.0, 2000.0, seed=7),
        "cl_dense": lambda: G.chung_lu(3000, 2.1, 30.0, 1500.0, seed=8),
        "er500": lambda: G.erdos_renyi_connected(500, 0.02, seed=9),
        "prism3": lambda: G.mirrored_prism(3),
    }[name]()


def test_hash_probe_matches_published_and_oracle():
    from oracle import oracle as O
    from paper_1412_0565_amd import cmg

    seq = cmg.cmg_hash_probe(1234567, -1, 5)
    assert [int(v) for v in seq] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                     4593380528125082431, 16408922859458223821]
    keys = cmg.cmg_hash_probe(14120565, 3, 4000)
    assert all(int(keys[v]) == O.hec_key(14120565, 3, v) for v in range(0, 4000, 37))


@pytest.mark.parametrize("name", ["path2", "path20", "K25", "grid5", "cycle101", "path1000", "K60", "star200",
                                  "grid100", "grid128", "grid_aniso", "grid3d_20", "rgg20k", "rgg60k",
                                  "cl30k", "cl_dense", "er500", "prism3"])
def test_fp64_parity(name):
    g = _named(name)
    say(f"[parity] {name} n={g.n} nnz={g.nnz}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)
    # the coarsest rule fixes the sign too
    assert float(np.dot(x, ref.y)) > 0


def test_hec_rounds_beyond_those_launched_ahead():
    """A path visited in ascending HEC key order with weights rising along
    it: each vertex's heaviest neighbour is the next one and every edge is a
    candidate, and a greedy round matches the first pair of the chain and
    kills the edge after it, so level 0 needs n / 2 rounds.  The rounds the
    setup launches before its first host check fall short; the matching is
    then finished and the aggregates formed again.  n is above the size the
    single-workgroup setup takes, so level 0 runs on the grid kernels."""
    from oracle import oracle as O

    n = 10000
    key = np.array([O.hec_key(14120565, 0, v) for v in range(n)], dtype=np.uint64)
    p = np.argsort(key, kind="stable")
    g = G.from_edges(n, p[:-1], p[1:], w=np.arange(1, n, dtype=float))
    say(f"[parity] key-ordered path n={g.n}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g)
    assert st.hec_rounds >= n // 2
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


def test_coarsest_fallback_start():
    # The ramp is orthogonal to the lambda_2 eigenspace of this graph (its
    # label reversal is an automorphism that fixes the eigenspace), so the
    # coarsest rule projects the hashed uniform start instead; a dense-only
    # solve must give the oracle's vector, sign included.
    g = _named("prism3")
    ref = oracle_of(g)
    z = np.arange(g.n) - (g.n - 1) / 2
    assert abs(float(ref.y @ z)) < 1e-12 * np.linalg.norm(z)  # the oracle took the fallback
    lam, x, st, levels, arrays = run_gpu(g)
    assert len(levels) == 1 and levels[0].k == -1
    assert np.allclose(x, ref.y, atol=1e-12)
    assert abs(lam - 1.0) <= 1e-12


@pytest.mark.parametrize("name,block_rows", [(nm, b) for nm in ["grid128", "grid3d_20", "rgg60k", "cl30k",
                                                                   "grid_aniso"] for b in (0, 1)]
                         + [("path1000", 1), ("star200", 1)])
def test_fp64_step_mode_parity(name, block_rows):
    # every grid level traversed by rows refined with one launch per PI step
    # (k_step_spmv + k_step_check, no grid barrier); block_rows=1 sends all
    # levels to the grid kernels, so coarse and tiny levels take this path too
    g = _named(name)
    say(f"[step mode] {name} n={g.n} nnz={g.nnz} block_rows={block_rows}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, step_mode=1, block_rows=block_rows)
    say(f"  step levels {[j for j, l in enumerate(levels) if l.step]} k {[l.k for l in levels]}")
    assert any(l.step for l in levels)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("name", ["grid128", "rgg60k", "grid3d_20"])
def test_mixed_step_mode(name):
    g = _named(name)
    say(f"[mixed step mode] {name}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, precision=1, mixed_min_nnz=1, step_mode=1, block_rows=1)
    assert any(l.step and l.fp32 for l in levels)
    assert abs(lam - ref.lam) <= MIXED_LAM_RTOL * ref.lam, (lam, ref.lam)
    assert st.residual < 10 * ref.residual + 1e-6
    assert abs(np.linalg.norm(x) - 1) < 1e-12


@pytest.mark.parametrize("step_mode", [0, -1])
def test_grid3d128_step_mode_default_and_off(step_mode):
    # 128^3 grid: by default its level 2 (depth 2, over 16 MB per step) runs
    # one launch per step; with step_mode=-1 every grid level keeps its
    # persistent launch.  Both match the oracle.
    g = G.grid3d(128)
    say(f"[step mode] grid3d128 step_mode={step_mode}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, step_mode=step_mode)
    say(f"  step levels {[j for j, l in enumerate(levels) if l.step]} k {[l.k for l in levels]}")
    assert any(l.step for l in levels) == (step_mode == 0)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("block_rows", [1, 1 << 30])
def test_block_and_grid_paths_agree_with_oracle(block_rows):
    g = G.grid2d(128, 128)
    say(f"[parity] grid128 block_rows={block_rows}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, block_rows=block_rows)
    assert all(l.in_block == (block_rows > 1) for l in levels[:-1])
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


def test_real_valued_weights():
    g = G.rgg(15000, 10.0, seed=3)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a = np.minimum(rows, g.col).astype(np.uint64)
    b = np.maximum(rows, g.col).astype(np.uint64)
    u = G.stream_uniform(11, 77, (a << np.uint64(32)) | b)
    g = G.CSR(g.n, g.row_ptr, g.col, 0.25 + 2.0 * u)
    say("[parity] real weights")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref, exact_g=False)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_seeds_and_options(seed):
    g = G.rgg(30000, 8.0, seed=seed)
    opts = dict(seed=1000 + seed, tol=1e-7 if seed == 2 else 1e-8, coarsest_n=40 if seed == 3 else 25)
    say(f"[parity] rgg30k seed={seed} {opts}")
    ref = oracle_of(g, **opts)
    lam, x, st, levels, arrays = run_gpu(g, **opts)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


def test_f32_input_weights():
    g = G.rgg(20000, 10.0, seed=12)
    g32 = g.astype(np.float32)
    say("[parity] f32 input")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g32)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("name", ["rgg60k", "grid128", "cl30k"])
def test_mixed_precision(name):
    g = _named(name)
    say(f"[mixed] {name}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, precision=1, mixed_min_nnz=1)
    assert any(l.fp32 for l in levels)
    say(f"  lambda {lam!r} oracle {ref.lam!r} rel {abs(lam - ref.lam) / ref.lam:.3e} "
        f"k {[l.k for l in levels]} oracle k {[l.k for l in ref.levels]}")
    assert abs(lam - ref.lam) <= MIXED_LAM_RTOL * ref.lam, (lam, ref.lam)
    assert st.residual < 10 * ref.residual + 1e-6
    assert abs(np.linalg.norm(x) - 1) < 1e-12


def test_deterministic_repeat():
    from paper_1412_0565_amd import cmg

    g = G.rgg(40000, 10.0, seed=2)
    say("[determinism] rgg40k")
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
        l1, x1, _ = F.solve()
        l2, x2, _ = F.solve()
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
        l3, x3, _ = F.solve()
    assert l1 == l2 == l3
    assert np.array_equal(x1, x2) and np.array_equal(x1, x3)


def test_coarsest_solve_reused_by_later_solves():
    """The dense coarsest solve runs on a handle's first solve only; later
    solves, solo or in a batch, and a graph that is one dense level give
    bitwise the results of the first solve."""
    from paper_1412_0565_amd import cmg

    for g in (G.complete(20), G.grid2d(40, 40)):
        with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
            l1, x1, _ = F.solve()
            l2, x2, _ = F.solve()
        assert l1 == l2 and np.array_equal(x1, x2), g.n
    ga, gb = G.rgg(20000, 10.0, seed=3), G.grid2d(90, 77, wx=2.0, wy=1.0)
    with cmg.Fiedler(ga.n, ga.row_ptr, ga.col, ga.w) as A, cmg.Fiedler(gb.n, gb.row_ptr, gb.col, gb.w) as B:
        la, xa, _ = A.solve()
        xs = [np.zeros(ga.n), np.zeros(gb.n)]
        lams, _ = cmg.cmg_fiedler_batch([A.handle, B.handle], xs)
        lb, xb, _ = B.solve()
        assert lams[0] == la and np.array_equal(xs[0], xa)
        assert lams[1] == lb and np.array_equal(xs[1], xb)
        ref = oracle_of(gb)
        assert abs(lb - ref.lam) <= 1e-9 * ref.lam


def test_device_tensors_and_torch_allocator():
    import torch
    from paper_1412_0565_amd import cmg

    g = G.grid2d(128, 128)
    say("[device] torch tensors")
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    w = torch.from_numpy(g.w).cuda()
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    alloc = cmg.torch_allocator()
    import ctypes as C

    opt = cmg.cmg_options_default(allocator=C.pointer(alloc),
                                  stream=C.c_void_p(torch.cuda.current_stream().cuda_stream))
    h = cmg.cmg_setup(g.n, rp, col, w, opt)
    try:
        lam, _ = cmg.cmg_fiedler(h, x)
        assert cmg.cmg_footprint(h) > 0
    finally:
        cmg.cmg_free(h)
    ref = oracle_of(g)
    assert cosine(x.cpu().numpy(), ref.y) >= 1 - 1e-10
    assert abs(lam - ref.lam) <= 1e-9 * ref.lam


@pytest.mark.parametrize("case", ["selfloop", "unsorted", "negative", "nan", "isolated", "badptr", "asym"])
def test_invalid_graphs(case):
    from paper_1412_0565_amd import cmg

    g = G.grid2d(10, 10)
    rp, col, w = g.row_ptr.copy(), g.col.copy(), g.w.copy()
    opts = {}
    if case == "selfloop":
        col[0] = 0
        exp = cmg.CMG_E_GRAPH
    elif case == "unsorted":
        col[0], col[1] = col[1], col[0]
        exp = cmg.CMG_E_GRAPH
    elif case == "negative":
        w[5] = -1.0
        exp = cmg.CMG_E_GRAPH
    elif case == "nan":
        w[7] = float("nan")
        exp = cmg.CMG_E_GRAPH
    elif case == "isolated":
        # vertex 0 loses its edges (and its neighbours lose vertex 0)
        e = g.edges()
        keep = (e[0] != 0) & (e[1] != 0)
        gg = G.from_edges(100, e[0][keep], e[1][keep])
        rp, col, w = gg.row_ptr, gg.col, gg.w
        exp = cmg.CMG_E_ISOLATED
    elif case == "badptr":
        rp[3] = rp[4] + 1
        exp = cmg.CMG_E_GRAPH
    elif case == "asym":
        w[3] = 2.0
        opts["validate_full"] = 1
        exp = cmg.CMG_E_GRAPH
    with pytest.raises(cmg.CmgError) as ei:
        cmg.cmg_setup(100, rp, col, w, cmg.cmg_options_default(**opts))
    assert ei.value.status == exp


def _grid_plus_edge(side):
    """A side x side grid with a separate two-vertex component: level 0 is
    valid, but the pair becomes one aggregate, a vertex with no neighbour
    on level 1."""
    g = G.grid2d(side, side)
    e = g.edges()
    n = g.n + 2
    return G.from_edges(n, np.concatenate([e[0], [g.n]]), np.concatenate([e[1], [g.n + 1]]))


@pytest.mark.parametrize("side", [40, 200])
def test_component_collapsing_to_an_isolated_coarse_vertex(side):
    """The oracle rejects the graph when HEC meets the vertex without a
    neighbour on level 1 (Algorithm 2 takes a heaviest neighbour); the GPU
    returns the same status, from the single-workgroup setup (side 40,
    level 1 of 534 vertices) and from the grid kernels (side 200, level 1 of
    over 13k vertices), after HEC ran on that level with the vertex naming
    itself."""
    from paper_1412_0565_amd import cmg

    g = _grid_plus_edge(side)
    assert oracle_of(g).status == "E_ISOLATED"
    say(f"[parity] grid {side}x{side} + edge: expecting CMG_E_ISOLATED")
    with pytest.raises(cmg.CmgError) as ei:
        cmg.cmg_setup(g.n, g.row_ptr, g.col, g.w, cmg.cmg_options_default())
    assert ei.value.status == cmg.CMG_E_ISOLATED
    # the library stays usable
    lam, x, st, levels, arrays = run_gpu(G.grid2d(30, 30))
    assert_fp64_parity(G.grid2d(30, 30), lam, x, st, levels, arrays, oracle_of(G.grid2d(30, 30)))


@pytest.mark.parametrize("case", ["valid", "unsorted", "duplicate", "range", "selfloop", "zero", "asym"])
def test_invalid_entry_deep_in_a_long_row(case):
    """Faults past the first lanes of the row check: the hub row of a
    40-vertex star holds 39 entries, each altered at positions 9-29."""
    from paper_1412_0565_amd import cmg

    g = G.star(40)
    rp, col, w = g.row_ptr.copy(), g.col.copy(), g.w.copy()
    hub = int(np.argmax(np.diff(rp)))
    a = int(rp[hub])
    assert rp[hub + 1] - a == 39
    opts = {}
    if case == "unsorted":
        col[a + 12], col[a + 13] = col[a + 13], col[a + 12]
    elif case == "duplicate":
        col[a + 20] = col[a + 19]
    elif case == "range":
        col[a + 29] = 40
    elif case == "selfloop":
        col[a + 9] = hub
    elif case == "zero":
        w[a + 17] = 0.0
    elif case == "asym":
        w[a + 17] = 3.0
        opts["validate_full"] = 1
    if case == "valid":
        opts["validate_full"] = 1
        h = cmg.cmg_setup(40, rp, col, w, cmg.cmg_options_default(**opts))
        cmg.cmg_free(h)
        return
    with pytest.raises(cmg.CmgError) as ei:
        cmg.cmg_setup(40, rp, col, w, cmg.cmg_options_default(**opts))
    assert ei.value.status == cmg.CMG_E_GRAPH


def test_maxit_warning():
    from paper_1412_0565_amd import cmg

    g = G.grid2d(64, 64)
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w, max_iters_per_level=3) as F:
        lam, x, st = F.solve()
        assert st.status == cmg.CMG_W_MAXIT
        assert all(l.k <= 3 for l in F.levels())
    ref = oracle_of(g, max_iters_per_level=3)
    assert cosine(x, ref.y) >= 1 - 1e-10


def test_courant_fischer_closed_forms():
    # r >= lambda_2 for closed-form spectra, independent of the oracle
    # (Courant-Fischer: the Rayleigh quotient of any vector orthogonal to 1
    # is at least lambda_2).  No upper bound follows from the paper at a
    # given tolerance: the stopping test compares successive iterates, and
    # Algorithm 1 itself (the oracle) stops at r = 1.0157, 1.0015 and 1.185
    # lambda_2 on these three graphs, so above that r is checked against
    # the oracle's value.
    for g, lam2 in [(G.grid2d(128, 128), 2 - 2 * math.cos(math.pi / 128)),
                    (G.grid3d(24), 2 - 2 * math.cos(math.pi / 24)),
                    (G.cycle(5000), 2 - 2 * math.cos(2 * math.pi / 5000))]:
        lam, x, st, levels, _ = run_gpu(g, want_levels=False)
        assert lam >= lam2 * (1 - 1e-12)
        ref = oracle_of(g)
        say(f"  n={g.n} r/lambda_2 gpu {lam / lam2:.6f} oracle {ref.lam / lam2:.6f}")
        assert abs(lam - ref.lam) <= 1e-9 * ref.lam


@pytest.fixture(scope="module")
def rgg1m():
    return G.workload("rgg1m")


@pytest.mark.parametrize("precision", [0, 1])
def test_fullsize_rgg1m_bench_config(rgg1m, precision):
    """The benchmark workload at full size, in the launch configuration
    bench.py times (torch allocator, torch stream, device arrays)."""
    import ctypes as C

    import torch
    from paper_1412_0565_amd import cmg

    g = rgg1m
    say(f"[fullsize] rgg1m n={g.n} nnz={g.nnz} precision={precision}")
    ref = oracle_of(g)
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
        arrays = [cmg.cmg_level_copy(h, j, levels[j].n, int(levels[j].nnz), with_agg=j < len(levels) - 1)
                  for j in range(len(levels))]
    finally:
        cmg.cmg_free(h)
    xh = x.cpu().numpy()
    say(f"  lambda {lam!r} oracle {ref.lam!r} k {[l.k for l in levels]} oracle {[l.k for l in ref.levels]}")
    if precision == 0:
        assert_fp64_parity(g, lam, xh, st, levels, arrays, ref)
    else:
        from gpu_compare import assert_hierarchy_equal

        assert_hierarchy_equal(g, ref, levels, arrays)
        assert abs(lam - ref.lam) <= MIXED_LAM_RTOL * ref.lam


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("name", ["grid128", "rgg20k", "cl30k", "cl_dense"])
def test_spmv_variants_against_oracle(variant, name):
    """Both SpMV traversals (lane groups per row, merge path) on every
    refinement level (block_rows=1 sends all levels to the grid kernels)."""
    g = _named(name)
    say(f"[variant] {name} variant={variant}")
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, spmv_variant=variant, block_rows=1)
    assert all(l.variant == variant for l in levels[:-1] if not l.in_block)
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


def _batch_graphs():
    return [("rgg20k", G.rgg(20000, 10.0, seed=5), {}),
            ("grid128", G.grid2d(128, 128), {}),
            ("cl30k", G.chung_lu(30000, 2.1, 16.0, 2000.0, seed=7), {"spmv_variant": 2}),
            ("path1000", G.path(1000), {}),
            ("K60", G.complete(60), {}),
            ("star200", G.star(200), {}),
            ("rgg60k_mixed", G.rgg(60000, 10.0, seed=6), {"precision": 1, "mixed_min_nnz": 1}),
            ("grid3d_20_tol", G.grid3d(20), {"tol": 1e-7, "block_rows": 500})]


def test_batch_equals_alone_bitwise():
    from paper_1412_0565_amd import cmg

    items = _batch_graphs()
    alone = []
    for name, g, opts in items:
        say(f"[batch] alone {name}")
        with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w, **opts) as F:
            lam, x, _ = F.solve()
        alone.append((lam, x))
    handles = [cmg.Fiedler(g.n, g.row_ptr, g.col, g.w, **opts) for _, g, opts in items]
    try:
        xs = [np.zeros(g.n) for _, g, _ in items]
        for rep in range(2):
            say(f"[batch] packed solve {rep}")
            lams, st = cmg.cmg_fiedler_batch([F.handle for F in handles], xs)
            for (name, g, _), (la, xa), lb, xb in zip(items, alone, lams, xs):
                assert la == lb, (name, la, lb)
                assert np.array_equal(xa, xb), name
    finally:
        for F in handles:
            F.close()


def test_batch_against_oracle():
    from paper_1412_0565_amd import cmg

    items = [it for it in _batch_graphs() if "mixed" not in it[0] and "tol" not in it[0]]
    handles = [cmg.Fiedler(g.n, g.row_ptr, g.col, g.w, **opts) for _, g, opts in items]
    try:
        xs = [np.zeros(g.n) for _, g, _ in items]
        stats = []
        lams, _ = cmg.cmg_fiedler_batch([F.handle for F in handles], xs, stats)
        for (name, g, _), lam, x, F in zip(items, lams, xs, handles):
            ref = oracle_of(g)
            levels = F.levels()
            assert [l.k for l in levels] == [l.k for l in ref.levels], name
            assert cosine(x, ref.y) >= 1 - 1e-10, name
            assert abs(lam - ref.lam) <= 1e-9 * ref.lam, name
    finally:
        for F in handles:
            F.close()


def test_batch_rejects_duplicates():
    from paper_1412_0565_amd import cmg

    g = G.grid2d(30, 30)
    with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
        with pytest.raises(cmg.CmgError):
            cmg.cmg_fiedler_batch([F.handle, F.handle])


@pytest.mark.parametrize("name", ["rgg20k", "rgg60k", "grid128", "grid3d_20", "cl30k"])
def test_grid_stage_is_bitwise_equal_to_global_reads(name):
    """Grid levels whose workgroup shares are staged in LDS (default) give
    bitwise the vector, lambda and step counts of the traversal that reads
    the level's arrays from global memory (grid_stage=0), FP64 and mixed;
    and both match the oracle."""
    g = _named(name)
    ref = oracle_of(g)
    for prec in (0, 1):
        res = {}
        for stage in (1, 0):
            lam, x, st, levels, arrays = run_gpu(g, want_levels=(prec == 0), precision=prec,
                                                 grid_stage=stage)
            res[stage] = (lam, np.asarray(x).copy(), [l.k for l in levels], arrays, levels, st)
        say(f"[parity] {name} precision={prec} grid levels "
            f"{[(j, l.grid) for j, l in enumerate(res[1][4]) if not l.in_block]} lam {res[1][0]!r}")
        assert res[1][0] == res[0][0], (name, prec)
        assert np.array_equal(res[1][1], res[0][1]), (name, prec)
        assert res[1][2] == res[0][2], (name, prec)
        if prec == 0:
            lam, x, k, arrays, levels, st = res[1]
            assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("name", ["rgg20k", "grid128", "grid3d_20", "er500", "star200", "cl30k"])
def test_block_register_rows_and_csr_agree_with_oracle(name):
    """Single-workgroup levels on register rows (default) and on the CSR
    traversal (block_regs=-1): both bit-exact in hierarchy and step counts
    against the oracle.  Graphs with short rows use register rows; rows up
    to twice a layout's slots keep the rest in an LDS list (a level of
    grid128, cl30k and er500 each); a hub row longer than that keeps its
    level on the CSR kernel."""
    g = _named(name)
    ref = oracle_of(g)
    for regs in (0, -1):
        lam, x, st, levels, arrays = run_gpu(g, block_regs=regs)
        lay = [(j, l.lanes, l.block_waves, l.block_regs, l.block_slots,
                int(np.diff(ref.levels[j].row_ptr).max())) for j, l in enumerate(levels) if l.in_block]
        say(f"[parity] {name} block_regs={regs} block levels "
            f"(j, lanes, waves, rows per group, slots, longest row) {lay}")
        if regs < 0:
            assert all(l.block_regs == 0 for l in levels)
        else:
            if name in ("rgg20k", "grid128", "grid3d_20"):
                assert any(l.block_regs > 0 for l in levels if l.in_block)
            if name in ("grid128", "cl30k", "er500"):
                # a level whose longest row exceeds lanes x slots
                assert any(r > 0 and ml > ln * sl for _, ln, _, r, sl, ml in lay)
            assert all(ml <= 2 * ln * sl for _, ln, _, r, sl, ml in lay if r > 0)
        assert_fp64_parity(g, lam, x, st, levels, arrays, ref)


@pytest.mark.parametrize("name", ["grid128", "rgg60k", "cl30k", "grid3d_20", "real_rgg"])
def test_galerkin_gather_and_sort_agree(name):
    # coarse rows formed per aggregate (default where aggregates are small:
    # in registers, the rows with many columns by a wavefront's sort), every
    # row by the wavefront's sort (galerkin=2) and by the radix sort over the
    # level (galerkin=1) sum in the same fine CSR order: all hierarchies
    # bitwise equal to the oracle's, real weights included
    if name == "real_rgg":
        g = G.rgg(40000, 10.0, seed=12, int_weights=False)
        rng = np.random.default_rng(3)
        r = rng.random(g.m) + 0.1
        u, v, _ = g.edges()
        g = G.from_edges(g.n, u, v, r)
    else:
        g = _named(name)
    ref = oracle_of(g)
    for mode in (0, 1, 2):
        lam, x, st, levels, arrays = run_gpu(g, galerkin=mode)
        # g = 2 max degree sums real weights in another order than the oracle
        assert_fp64_parity(g, lam, x, st, levels, arrays, ref, exact_g=name != "real_rgg")


@pytest.mark.parametrize("name,level", [("grid128", 0), ("rgg60k", 0), ("rgg60k", 1), ("grid3d_20", 0)])
def test_barrier_fallback_matches_oracle(name, level):
    # the first attempt raises the barrier's abort flag from the host before
    # the level's persistent launch (every kernel then exits normally); the
    # call re-runs the persistent levels one launch per step and returns the
    # oracle's result, step counts included
    g = _named(name)
    ref = oracle_of(g)
    lam, x, st, levels, arrays = run_gpu(g, test_abort_level=level)
    say(f"[fallback] {name} level {level}: fallback={st.fallback} k {[l.k for l in levels]}")
    assert not levels[level].in_block and not levels[level].step
    assert st.fallback == 1
    assert_fp64_parity(g, lam, x, st, levels, arrays, ref)
    lam2, x2, st2, _, _ = run_gpu(g, want_levels=False)
    assert st2.fallback == 0


def test_barrier_fallback_mixed():
    g = _named("rgg60k")
    ref = oracle_of(g)
    lam, x, st, levels, _ = run_gpu(g, want_levels=False, test_abort_level=0, precision=1, mixed_min_nnz=1)
    assert st.fallback == 1
    assert abs(lam - ref.lam) <= MIXED_LAM_RTOL * ref.lam


@pytest.mark.parametrize("name", ["grid128", "grid3d_20", "rgg60k", "grid_aniso", "cl30k"])
@pytest.mark.parametrize("mode", ["grid", "step", "mixed"])
def test_narrow_weight_storage_is_bitwise_fp64_storage(name, mode):
    # the grid and step kernels read no weights where all are 1, an 8- or
    # 16-bit copy where all are integers up to 255 or 65535 and an FP32 copy
    # where all are exact in FP32: the values are the same doubles, so step
    # counts, lambda and the vector equal FP64 storage bit for bit, and both
    # match the oracle
    g = _named(name)
    ref = oracle_of(g)
    kw = {"block_rows": 1}
    if mode == "step":
        kw["step_mode"] = 1
    if mode == "mixed":
        kw.update(precision=1, mixed_min_nnz=1)
    runs = {}
    for ws in (0, 1):
        lam, x, st, levels, _ = run_gpu(g, want_levels=False, weight_storage=ws, **kw)
        runs[ws] = (lam, x, [l.k for l in levels], [l.weights for l in levels])
    say(f"[weights] {name} {mode}: storage {runs[0][3]} vs {runs[1][3]} k {runs[0][2]}")
    assert runs[0][2] == runs[1][2]
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])
    unit = bool(np.all(g.w == 1.0))
    if mode != "mixed":
        assert all(w == 0 for w in runs[1][3])
        assert (runs[0][3][0] == 2) == unit, runs[0][3]
        if name in ("rgg60k", "grid_aniso"):
            # integer weights 1..8 and 1..2: the 8-bit copy
            assert runs[0][3][0] == 3, runs[0][3]
        if name in ("rgg60k", "cl30k"):
            # coarse integer weights above 255 (at most 65535): the 16-bit copy
            assert 4 in runs[0][3], runs[0][3]
        assert [l.k for l in ref.levels] == runs[0][2]
    elif name in ("rgg60k", "grid_aniso"):
        # FP32 iterates read the 8-bit copy of small integer weights too
        assert runs[0][3][0] == 3, runs[0][3]
    lam_ref = ref.lam
    assert abs(runs[0][0] - lam_ref) <= (1e-5 if mode == "mixed" else 1e-9) * abs(lam_ref)
