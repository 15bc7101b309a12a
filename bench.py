#!/usr/bin/env python3
"""Benchmark: Fiedler solves/s of the cascadic multigrid path on one MI355X.

One step = one whole solve of the workload: cmg_setup (validation, HEC
coarsening, Galerkin hierarchy) + cmg_fiedler (coarsest solve, cascadic
power-iteration refinement, Rayleigh quotient and residual) + cmg_free,
with the input graph already resident in HBM.

Default workload: the 3D 256^3 seven-point grid graph (16.8M vertices,
100M stored entries, unit weights given as FP32), solved in FP64: the
largest configuration on one GPU.  The same graph is also solved with the
mixed FP32/FP64 path and with a resident hierarchy (cmg_fiedler only);
those figures are reported beside the main value.  The roofline entry
covers the finest-level power-iteration launch (the SpMV hot loop), timed
with HIP events on the library's stream; `hbm_levels` adds up every level
whose matrix (nnz (4 + s_v) bytes) exceeds the 256 MiB last-level cache.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import platform
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Fiedler solves/s + SpMV HBM GB/s vs peak; p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rgg1m": "random geometric graph: 1M points uniform in the unit square, radius for mean degree 10, "
             "largest connected component, integer weights 1..8, CSR int32/float64",
    "grid128": "2D 128x128 5-point grid graph, unit weights, CSR int32/float64",
    "grid3d256": "3D 256^3 7-point grid graph, unit weights, CSR int32/float32",
    "chunglu4m": "Chung-Lu power-law graph, 4M vertices, exponent 2.1, mean degree 16, max degree 50k, "
                 "largest connected component, unit weights, CSR int32/float32",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def solve_once(cmg, g_dev, n, opt, x):
    rp, col, w = g_dev
    h = cmg.cmg_setup(n, rp, col, w, opt)
    st = cmg.cmg_stats()
    st.struct_size = C.sizeof(cmg.cmg_stats)
    try:
        lam, _ = cmg.cmg_fiedler(h, x, st)
        levels = cmg.cmg_level_info(h)
    finally:
        cmg.cmg_free(h)
    return lam, st, levels


def measured_traffic(workload, level0):
    """HBM bytes per level-0 refinement launch from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a copy kernel), or None if
    there is none for this workload and these kernel sources."""
    from paper_1412_0565_amd.profsum import kernel_source_hash

    path = os.path.join(ROOT, "profiles", f"{workload}_level0_refine_hbm_counters.md")
    try:
        kv = {}
        for line in open(path):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    except OSError:
        return None, None
    if kv.get("kernel sources") != kernel_source_hash() or int(kv.get("level-0 k", -1)) != level0.k:
        return None, f"{os.path.relpath(path, ROOT)} (stale: taken on other kernel sources)"
    return int(float(kv["HBM bytes per launch"])), os.path.relpath(path, ROOT)


def setup_bytes(levels):
    """Compulsory traffic of cmg_setup: for each level that is coarsened,
    the row pass (row pointers, columns, FP64 weights unless all are 1),
    the Galerkin read (row pointers, columns, the aggregate of every column,
    the weights, the aggregate of every vertex) and the coarse level's CSR
    written (row pointers, columns, FP64 weights).  HEC rounds, scans and
    member lists are not counted, so the fraction is an upper bound on how
    close setup runs to HBM."""
    b = 0
    for j in range(len(levels) - 1):
        L, C = levels[j], levels[j + 1]
        sw = 0 if L.weights == 2 else 8
        b += 4 * (L.n + 1) + L.nnz * (4 + sw)
        b += 4 * (L.n + 1) + L.nnz * (8 + sw) + 4 * L.n
        b += 4 * (C.n + 1) + 12 * C.nnz
    return b


def setup_roofline(levels, setup_ms):
    sb = setup_bytes(levels)
    gbs = sb / (setup_ms * 1e-3) / 1e9
    return {"bound": "hbm", "bytes": sb, "ms": round(setup_ms, 3), "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "counted": "row pass, Galerkin read and coarse CSR write of every coarsened level"}


def launch_bytes(levels, j=0):
    """Algorithmic bytes of the level-j refinement launch: k PI steps of
    4(n+1) + nnz(4+s_v) + 2 s_x n, plus the prolongation (agg read, coarse
    gather, write) and the deflation pass over the start vector."""
    L = levels[j]
    sx = 4 if L.fp32 else 8
    nc = levels[j + 1].n if j + 1 < len(levels) else 0
    prol = 4 * L.n + sx * nc + 2 * sx * L.n
    return L.k * L.bytes_per_iter + prol


def serve_leg(args):
    """Served stream shaped like the paper-derived serving workload: requests
    drawn from a seeded pool of graphs (sizes log-uniform over 1k-1M
    vertices; 2D grids, RGGs, Chung-Lu; integer weights), Poisson arrivals
    at 0.7x the closed-loop throughput of the plain FP64 one-at-a-time path.
    The same stream is replayed through the server twice: plain FP64 with
    batches of one in arrival order, and mixed precision with cost-aware
    continuous batching (up to 64 graphs per packed launch).  Hierarchies
    stay resident (LRU) under an HBM budget small enough for admission to
    bind.  A no-repeat variant sends every pool graph once (every request
    builds its hierarchy)."""
    import numpy as np

    from paper_1412_0565_amd import cmg
    from paper_1412_0565_amd import graphs as G
    from paper_1412_0565_amd.serve import CmgBackend, Request, Server, latency_summary, replay

    t0 = time.time()
    pool = G.serve_pool(args.serve_pool)
    log(f"[serve] pool of {len(pool)} graphs generated in {time.time() - t0:.1f}s "
        f"(n {min(g.n for _, g in pool)}..{max(g.n for _, g in pool)})")
    rng = np.random.default_rng(20260101)
    picks = rng.integers(0, len(pool), args.serve_requests)
    # closed-loop throughput of the plain FP64 path: setup + solve, one at a time
    t = time.perf_counter()
    m = min(len(pool), 16)
    for i in range(m):
        _, g = pool[int(picks[i])]
        t1 = time.perf_counter()
        with cmg.Fiedler(g.n, g.row_ptr, g.col, g.w) as F:
            F.solve()
        log(f"[serve] closed loop {i + 1}/{m}: n={g.n} nnz={g.nnz} {1e3 * (time.perf_counter() - t1):.1f} ms")
    x_fp64 = m / (time.perf_counter() - t)
    qps = 0.7 * x_fp64
    budget = int(args.serve_budget_gb * (1 << 30))
    backend = CmgBackend()
    res = {"pool": len(pool), "requests": args.serve_requests,
           "requests_note": f"{args.serve_requests} requests per path (the serving workload names 10,000; "
                            f"reduced to keep the run to minutes)",
           "qps": round(qps, 2), "closed_loop_fp64_solves_per_s": round(x_fp64, 2), "budget_bytes": budget}
    legs = [("fp64_sequential", 0, 1, "fifo", list(picks)), ("mixed_batched", 1, 64, "cost", list(picks)),
            ("mixed_batched_no_repeat", 1, 64, "cost", list(range(min(args.serve_norepeat, len(pool)))))]
    for label, prec, maxb, policy, order in legs:
        stream = [Request(i, pool[int(p)][0], pool[int(p)][1].n, pool[int(p)][1].row_ptr, pool[int(p)][1].col,
                          pool[int(p)][1].w, precision=prec) for i, p in enumerate(order)]
        srv = Server(backend, budget_bytes=budget, max_batch=maxb, policy=policy)
        log(f"[serve] {label}: {len(stream)} requests at {qps:.1f}/s")
        try:
            replay(srv, stream, qps=qps, seed=7,
                   progress=lambda d, tot: log(f"[serve] {label}: {d}/{tot} completed"), every=100)
        finally:
            srv.close()
        summ = latency_summary(stream)
        summ["requests"] = len(stream)
        summ["mean_batch"] = round(float(np.mean(srv.batches)), 2) if srv.batches else 0.0
        summ["max_batch"] = int(max(srv.batches)) if srv.batches else 0
        summ["peak_reserved_bytes"] = int(srv.peak)
        summ["evictions"] = int(srv.evictions)
        summ["failed"] = sum(r.status != "done" for r in stream)
        for r in stream:
            if r.status != "done":
                log(f"[serve] {label}: request {r.rid} (n={r.n}) {r.status}: {r.error}")
        res[label] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
        log(f"[serve] {label}: {res[label]}")
    return res


def extras_leg(args, g, g_dev, opts):
    """The next rows built beside the hot path, on the same workload:
    Algorithm 4's fixed schedule replayed from a captured HIP graph, heavy
    edge matching against HEC, several eigenpairs, recursive bisection."""
    import numpy as np
    import torch

    from paper_1412_0565_amd import cmg
    from paper_1412_0565_amd import graphs as G

    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    out = {}

    def resident_rate(opt, reps=10):
        h = cmg.cmg_setup(g.n, *g_dev, opt)
        try:
            for _ in range(2):
                cmg.cmg_fiedler(h, x)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                lam, _ = cmg.cmg_fiedler(h, x)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t) / reps
            st = cmg.cmg_stats()
            st.struct_size = C.sizeof(cmg.cmg_stats)
            cmg.cmg_fiedler(h, x, st)
            levels = cmg.cmg_level_info(h)
            return el, lam, st, levels, st.setup_ms
        finally:
            cmg.cmg_free(h)

    # fixed schedule k_j = ceil(3 * 1.6^j), graph replay
    el, lam, st, levels, _ = resident_rate(opts(precision=cmg.CMG_FP64, fixed_k0=3, fixed_beta=1.6, graph=1))
    out["fixed_schedule"] = {"k0": 3, "beta": 1.6, "steps": [L.k for L in levels],
                             "resident_solves_per_s": round(1.0 / el, 2), "lambda": lam,
                             "residual": st.residual, "graph_replay": True}
    log(f"[extras] fixed schedule: {1.0 / el:.2f} resident solves/s lambda {lam:.12e} residual {st.residual:.3e}")
    # coarsening ablation: HEC against heavy edge matching
    abl = {}
    for label, cz in [("hec", 0), ("hem", 1)]:
        t = time.perf_counter()
        h = cmg.cmg_setup(g.n, *g_dev, opts(precision=cmg.CMG_FP64, coarsen=cz))
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t)
        try:
            st = cmg.cmg_stats()
            st.struct_size = C.sizeof(cmg.cmg_stats)
            t = time.perf_counter()
            lam, _ = cmg.cmg_fiedler(h, x, st)
            solve_ms = 1e3 * (time.perf_counter() - t)
            levels = cmg.cmg_level_info(h)
        finally:
            cmg.cmg_free(h)
        abl[label] = {"levels": len(levels), "sizes": [L.n for L in levels][:6], "setup_ms": round(setup_ms, 2),
                      "solve_ms": round(solve_ms, 2), "lambda": lam, "residual": st.residual}
        log(f"[extras] {label}: {len(levels)} levels setup {setup_ms:.1f} ms solve {solve_ms:.1f} ms "
            f"lambda {lam:.10e} residual {st.residual:.3e}")
    out["coarsening_ablation"] = abl
    # several eigenpairs
    h = cmg.cmg_setup(g.n, *g_dev, opts(precision=cmg.CMG_FP64))
    try:
        X = torch.zeros(4 * g.n, dtype=torch.float64, device="cuda")
        cmg.cmg_fiedler_block(h, 4, X)
        torch.cuda.synchronize()
        t = time.perf_counter()
        lams, res, steps, _ = cmg.cmg_fiedler_block(h, 4, X)
        torch.cuda.synchronize()
        out["block_p4"] = {"ms": round(1e3 * (time.perf_counter() - t), 2), "lambdas": [float(v) for v in lams],
                           "residuals": [float(v) for v in res], "steps": steps}
        log(f"[extras] block p=4: {out['block_p4']['ms']} ms lambdas {lams}")
        del X
    finally:
        cmg.cmg_free(h)
    # recursive spectral bisection, 16 parts
    part = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, cut = cmg.cmg_bisect(g.n, *g_dev, 4, part=part, opt=opts(precision=cmg.CMG_FP64))
    torch.cuda.synchronize()
    sizes = torch.bincount(part.long(), minlength=16).cpu().numpy()
    out["bisection_16"] = {"ms": round(1e3 * (time.perf_counter() - t), 1), "cut": cut,
                           "part_sizes_min_max": [int(sizes.min()), int(sizes.max())]}
    log(f"[extras] bisection into 16: {out['bisection_16']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid3d256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=0,
                    help="oracle solves for the CPU baseline (0: about 10-30 s of work for the workload)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serve-pool", type=int, default=100)
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-norepeat", type=int, default=100)
    ap.add_argument("--serve-budget-gb", type=float, default=2.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="finish with one device-to-device copy of this many MiB (the reference kernel that "
                         "scales the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; the solver has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1412_0565_amd import cmg
    from paper_1412_0565_amd import graphs as G

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cmg.lib()

    t0 = time.time()
    g = G.workload(args.workload)
    log(f"[bench] workload {args.workload}: n={g.n} nnz={g.nnz} (generated in {time.time() - t0:.1f}s)")
    g_dev = (torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(), torch.from_numpy(g.w).cuda())
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    alloc = cmg.torch_allocator()

    def opts(**kw):
        return cmg.cmg_options_default(stream=C.c_void_p(stream.cuda_stream), allocator=C.pointer(alloc), **kw)

    fp64_opt = opts(precision=cmg.CMG_FP64)
    mixed_opt = opts(precision=cmg.CMG_MIXED)

    def timed(opt, steps, warmup, label):
        for _ in range(warmup):
            solve_once(cmg, g_dev, g.n, opt, x)
        torch.cuda.synchronize()
        pis, ks, byts, lams, setups = [], [], [], [], []
        t = time.perf_counter()
        for i in range(steps):
            lam, st, levels = solve_once(cmg, g_dev, g.n, opt, x)
            pis.append(levels[0].pi_ms)
            ks.append(levels[0].k)
            byts.append(launch_bytes(levels, 0))
            lams.append(lam)
            setups.append(st.setup_ms)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        log(f"[bench] {label}: {steps} solves in {el:.3f}s ({steps / el:.2f} solves/s), lambda={lams[-1]:.12e} "
            f"k0={ks[-1]} level-0 PI {statistics.mean(pis):.3f} ms")
        return el, pis, ks, byts, lams, setups, st, levels

    el, pis, ks, byts, lams, setups, st, levels = timed(fp64_opt, args.steps, args.warmup, "fp64 end-to-end")
    for j, L in enumerate(levels):
        log(f"[bench]   level {j}: n={L.n} nnz={L.nnz} k={L.k} lanes={L.lanes} grid={L.grid} "
            f"block={L.in_block} fp32={L.fp32} pi_ms={L.pi_ms:.4f}")
    value = args.steps / el
    ms_per_step = 1000.0 * el / args.steps

    # resident hierarchy: cmg_fiedler only
    h = cmg.cmg_setup(g.n, *g_dev, fp64_opt)
    try:
        for _ in range(args.warmup):
            cmg.cmg_fiedler(h, x)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            cmg.cmg_fiedler(h, x)
        torch.cuda.synchronize()
        el_res = time.perf_counter() - t
        fp = cmg.cmg_footprint(h)
    finally:
        cmg.cmg_free(h)

    mixed = None
    if not args.no_mixed:
        el_m, pis_m, ks_m, byts_m, lams_m, _, st_m, levels_m = timed(mixed_opt, args.steps, args.warmup,
                                                                     "mixed end-to-end")
        mixed = {
            "solves_per_s": round(args.steps / el_m, 3),
            "ms_per_step": round(1000.0 * el_m / args.steps, 3),
            "lambda": lams_m[-1],
            "lambda_rel_diff_vs_fp64": abs(lams_m[-1] - lams[-1]) / abs(lams[-1]),
            "residual": st_m.residual,
            "finest_pi_ms": round(statistics.mean(pis_m), 4),
            "finest_pi_GBps": round(statistics.mean(byts_m) / (statistics.mean(pis_m) * 1e-3) / 1e9, 1),
            "fp32_levels": [j for j, L in enumerate(levels_m) if L.fp32],
        }

    pi_ms = statistics.mean(pis)
    bytes_launch = statistics.mean(byts)
    achieved = bytes_launch / (pi_ms * 1e-3) / 1e9
    # levels whose matrix alone exceeds the 256 MiB last-level cache stream
    # from HBM on every step: their algorithmic bytes over their launch time
    hbm_j = [j for j, L in enumerate(levels)
             if not L.in_block and L.k > 0 and L.nnz * (4 + (4 if L.fp32 else 8)) > (256 << 20)]
    hbm_levels = None
    if hbm_j:
        hb = sum(launch_bytes(levels, j) for j in hbm_j)
        ht = sum(levels[j].pi_ms for j in hbm_j)
        hbm_levels = {"levels": hbm_j, "bytes": int(hb), "ms": round(ht, 4),
                      "achieved": round(hb / (ht * 1e-3) / 1e9, 1),
                      "frac": round(hb / (ht * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "per_level_GBps": [round(launch_bytes(levels, j) / (levels[j].pi_ms * 1e-3) / 1e9, 1)
                                         for j in hbm_j]}
    traffic, traffic_src = measured_traffic(args.workload, levels[0])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": traffic_src,
                "kernel": (f"k_refine_rows<{levels[0].lanes}, double, {levels[0].weights}>" if levels[0].variant != 2
                           else f"k_refine_merge<double, {levels[0].weights}>")
                          + f" on level 0 (prolongation, deflation, {ks[-1]} PI steps)",
                "bytes_per_launch": int(bytes_launch), "avg_launch_ms": round(pi_ms, 4),
                "pi_steps_per_launch": ks[-1], "hbm_levels": hbm_levels}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        O.lib()
        reps = args.cpu_repeats if args.cpu_repeats > 0 else {"rgg1m": 8, "grid128": 200}.get(args.workload, 1)
        t = time.perf_counter()
        for _ in range(reps):
            r = O.cmg(g, keep_levels=False)
        el_cpu = time.perf_counter() - t
        cpu = {"value": round(reps / el_cpu, 4), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full FP64 solves of the same {args.workload} graph by the single-threaded C "
                         f"oracle ({el_cpu:.1f}s)",
               "cpu_model": cpu_model(), "host_nproc": os.cpu_count(),
               "lambda": r.lam, "lambda_rel_diff_gpu": abs(r.lam - lams[-1]) / abs(r.lam)}
        log(f"[bench] cpu oracle: {reps} solves in {el_cpu:.2f}s")

    extras = None if args.no_extras else extras_leg(args, g, g_dev, opts)
    serve = None if args.no_serve else serve_leg(args)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "name": args.workload, "n": g.n, "nnz": g.nnz,
                   "levels": [L.n for L in levels], "pi_steps": [L.k for L in levels],
                   "tol": 1e-8, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "resident_solves_per_s": round(args.steps / el_res, 3),
        "setup_ms": round(statistics.mean(setups), 3),
        "setup_roofline": setup_roofline(levels, statistics.mean(setups)),
        "lambda": lams[-1],
        "residual": st.residual,
        "footprint_bytes": fp,
        "mixed": mixed,
        "extras": extras,
        "serve": serve,
    }
    if args.copy_mib > 0:
        nb = args.copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] reference copy: {nb} bytes read, {nb} bytes written")
        # a second reference with plain vector loads and stores: an
        # elementwise kernel reading and writing the same byte counts
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] reference elementwise add: {nb} bytes read, {nb} bytes written")
        del src, dst
    # every handle is freed; leave nothing queued or cached on the device
    # for the runtime's exit-time teardown
    del g_dev, x
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
