"""ctypes wrapper around the plain-C FP64 CPU oracle (``cmg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product library.
The wrapper only marshals arguments; all arithmetic is in the C file.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")

STATUS = {0: "OK", 1: "E_ARG", 2: "E_GRAPH", 3: "E_ISOLATED", 4: "E_OOM", 6: "W_MAXIT"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_splitmix64_sequence.argtypes = [C.c_uint64, C.c_int32, _u64p]
        L.orc_hec_key.restype = C.c_uint64
        L.orc_hec_key.argtypes = [C.c_uint64, C.c_int32, C.c_int32]
        L.orc_uniform.restype = C.c_double
        L.orc_uniform.argtypes = [C.c_uint64, C.c_int32]
        L.orc_laplacian_apply.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_gershgorin.restype = C.c_double
        L.orc_gershgorin.argtypes = [C.c_int32, _i32p, _f64p]
        L.orc_validate.restype = C.c_int
        L.orc_validate.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _f64p]
        L.orc_heaviest.restype = C.c_int
        L.orc_heaviest.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p]
        L.orc_hec_order.restype = C.c_int32
        L.orc_hec_order.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p, _i32p, _u8p]
        L.orc_hec.restype = C.c_int32
        L.orc_hec.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_uint64, C.c_int32, _i32p, _u8p]
        L.orc_galerkin.restype = C.c_int64
        L.orc_galerkin.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p, C.c_int32,
                                   C.POINTER(C.POINTER(C.c_int32)), C.POINTER(C.POINTER(C.c_int32)),
                                   C.POINTER(C.POINTER(C.c_double))]
        L.orc_jacobi.restype = C.c_int
        L.orc_jacobi.argtypes = [C.c_int32, _f64p, _f64p, _f64p]
        L.orc_coarsest_dense.restype = C.c_int
        L.orc_coarsest_dense.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_uint64, _f64p,
                                         C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.orc_pi.restype = C.c_int32
        L.orc_pi.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_double, _f64p, C.c_double, C.c_int32,
                             _f64p, C.POINTER(C.c_double)]
        L.orc_rq_residual.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.orc_hem_order.restype = C.c_int32
        L.orc_hem_order.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _i32p, _i32p, _u8p]
        L.orc_hem.restype = C.c_int32
        L.orc_hem.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_uint64, C.c_int32, _i32p, _u8p]
        L.orc_fixed_steps.restype = C.c_int32
        L.orc_fixed_steps.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_int32]
        L.orc_pi_fixed.restype = None
        L.orc_pi_fixed.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_double, _f64p, C.c_int32, _f64p,
                                   C.POINTER(C.c_double)]
        L.orc_cmg_ex.restype = C.c_void_p
        L.orc_cmg_ex.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _f64p, C.c_double, C.c_int32,
                                 C.c_int32, C.c_uint64, C.c_int32, C.c_int32, C.c_double, C.c_int32]
        L.orc_cmg_block.restype = C.c_void_p
        L.orc_cmg_block.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _f64p, C.c_double, C.c_int32,
                                    C.c_int32, C.c_uint64, C.c_int32, C.c_int32, C.c_double, C.c_int32]
        L.orc_block_free.argtypes = [C.c_void_p]
        for nm, rt in [("orc_block_status", C.c_int32), ("orc_block_nlevels", C.c_int32)]:
            getattr(L, nm).restype = rt
            getattr(L, nm).argtypes = [C.c_void_p]
        for nm, rt in [("orc_block_k", C.c_int32), ("orc_block_lambda", C.c_double),
                       ("orc_block_residual", C.c_double), ("orc_block_coarse", C.c_double)]:
            getattr(L, nm).restype = rt
            getattr(L, nm).argtypes = [C.c_void_p, C.c_int32]
        L.orc_block_copy_x.argtypes = [C.c_void_p, C.c_int32, _f64p]
        L.orc_coarsest_block.restype = C.c_int
        L.orc_coarsest_block.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_uint64, C.c_int32, _f64p, _f64p]
        L.orc_block_pi.restype = C.c_int32
        L.orc_block_pi.argtypes = [C.c_int32, _i32p, _i32p, _f64p, C.c_double, C.c_int32, _f64p, C.c_double,
                                   C.c_int32, C.c_int32, _f64p, C.POINTER(C.c_double)]
        L.orc_components.restype = C.c_int32
        L.orc_components.argtypes = [C.c_int32, _i32p, _i32p, _i32p]
        L.orc_rsb.restype = C.c_int
        L.orc_rsb.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _f64p, C.c_int32, _i32p]
        L.orc_cmg.restype = C.c_void_p
        L.orc_cmg.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _f64p, C.c_double, C.c_int32,
                              C.c_int32, C.c_uint64, C.c_int32]
        L.orc_free.argtypes = [C.c_void_p]
        for nm, rt in [("orc_res_status", C.c_int32), ("orc_res_nlevels", C.c_int32),
                       ("orc_res_collapsed", C.c_int32), ("orc_res_coarse_mult", C.c_int32)]:
            getattr(L, nm).restype = rt
            getattr(L, nm).argtypes = [C.c_void_p]
        for nm in ["orc_res_lambda", "orc_res_residual", "orc_res_coarse_lambda2"]:
            getattr(L, nm).restype = C.c_double
            getattr(L, nm).argtypes = [C.c_void_p]
        for nm, rt in [("orc_res_level_n", C.c_int32), ("orc_res_level_nnz", C.c_int64),
                       ("orc_res_level_g", C.c_double), ("orc_res_level_k", C.c_int32),
                       ("orc_res_level_margin", C.c_double)]:
            getattr(L, nm).restype = rt
            getattr(L, nm).argtypes = [C.c_void_p, C.c_int32]
        L.orc_res_copy_level.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
        L.orc_res_copy_y.argtypes = [C.c_void_p, _f64p]
        _lib = L
    return _lib


def _csr_args(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.float64)
    return rp, col, w


# ------------------------------------------------------------------ pieces

@dataclasses.dataclass
class Graph:
    """Plain CSR container returned by the oracle (n, row_ptr, col, w)."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def mix64(x: int) -> int:
    return int(lib().orc_mix64(x))


def splitmix64_sequence(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    lib().orc_splitmix64_sequence(seed, count, out)
    return out


def hec_key(seed: int, level: int, v: int) -> int:
    return int(lib().orc_hec_key(seed, level, v))


def uniform(seed: int, i: int) -> float:
    return float(lib().orc_uniform(seed, i))


def laplacian_apply(g, x):
    rp, col, w = _csr_args(g)
    y = np.zeros(g.n)
    lib().orc_laplacian_apply(g.n, rp, col, w, np.ascontiguousarray(x, dtype=np.float64), y)
    return y


def gershgorin(g) -> float:
    rp, col, w = _csr_args(g)
    return float(lib().orc_gershgorin(g.n, rp, w))


def validate(g) -> str:
    rp, col, w = _csr_args(g)
    return STATUS[lib().orc_validate(g.n, int(rp[-1]), rp, col, w)]


def heaviest(g) -> np.ndarray:
    rp, col, w = _csr_args(g)
    h = np.zeros(g.n, dtype=np.int32)
    st = lib().orc_heaviest(g.n, rp, col, w, h)
    if st != 0:
        raise ValueError(STATUS[st])
    return h


def hec_order(g, order):
    rp, col, w = _csr_args(g)
    agg = np.zeros(g.n, dtype=np.int32)
    sd = np.zeros(g.n, dtype=np.uint8)
    c = lib().orc_hec_order(g.n, rp, col, w, np.ascontiguousarray(order, dtype=np.int32), agg, sd)
    if c < 0:
        raise ValueError("hec failed")
    return agg, sd.astype(bool), int(c)


def hec(g, seed: int, level: int):
    rp, col, w = _csr_args(g)
    agg = np.zeros(g.n, dtype=np.int32)
    sd = np.zeros(g.n, dtype=np.uint8)
    c = lib().orc_hec(g.n, rp, col, w, seed, level, agg, sd)
    if c < 0:
        raise ValueError("hec failed")
    return agg, sd.astype(bool), int(c)


def hem_order(g, order):
    rp, col, w = _csr_args(g)
    agg = np.zeros(g.n, dtype=np.int32)
    sd = np.zeros(g.n, dtype=np.uint8)
    c = lib().orc_hem_order(g.n, rp, col, w, np.ascontiguousarray(order, dtype=np.int32), agg, sd)
    if c < 0:
        raise ValueError("hem failed")
    return agg, sd.astype(bool), int(c)


def hem(g, seed: int, level: int):
    rp, col, w = _csr_args(g)
    agg = np.zeros(g.n, dtype=np.int32)
    sd = np.zeros(g.n, dtype=np.uint8)
    c = lib().orc_hem(g.n, rp, col, w, seed, level, agg, sd)
    if c < 0:
        raise ValueError("hem failed")
    return agg, sd.astype(bool), int(c)


def fixed_steps(k0: int, beta: float, j: int, max_iters: int = 100000) -> int:
    return int(lib().orc_fixed_steps(k0, beta, j, max_iters))


def pi_fixed(g, y0, steps: int, gval: float | None = None):
    rp, col, w = _csr_args(g)
    if gval is None:
        gval = gershgorin(g)
    y = np.zeros(g.n)
    utv = C.c_double()
    lib().orc_pi_fixed(g.n, rp, col, w, gval, np.ascontiguousarray(y0, dtype=np.float64), steps, y,
                       C.byref(utv))
    return y, float(utv.value)


def galerkin(g, agg, nc):
    """Returns (row_ptr, col, w) of the coarse graph."""
    rp, col, w = _csr_args(g)
    prp = C.POINTER(C.c_int32)()
    pcol = C.POINTER(C.c_int32)()
    pw = C.POINTER(C.c_double)()
    nz = lib().orc_galerkin(g.n, rp, col, w, np.ascontiguousarray(agg, dtype=np.int32), nc,
                            C.byref(prp), C.byref(pcol), C.byref(pw))
    if nz < 0:
        raise MemoryError
    crp = np.ctypeslib.as_array(prp, shape=(nc + 1,)).copy()
    ccol = np.ctypeslib.as_array(pcol, shape=(max(nz, 1),))[:nz].copy()
    cw = np.ctypeslib.as_array(pw, shape=(max(nz, 1),))[:nz].copy()
    libc = C.CDLL(None)
    libc.free.argtypes = [C.c_void_p]
    for p in (prp, pcol, pw):
        libc.free(C.cast(p, C.c_void_p))
    return Graph(nc, crp, ccol, cw)


def jacobi(A):
    A = np.array(A, dtype=np.float64, copy=True, order="C")
    n = A.shape[0]
    V = np.zeros((n, n))
    ev = np.zeros(n)
    sweeps = lib().orc_jacobi(n, A.reshape(-1), V.reshape(-1), ev)
    return ev, V, int(sweeps)


def coarsest_dense(g, seed: int = 14120565):
    rp, col, w = _csr_args(g)
    y = np.zeros(g.n)
    lam = C.c_double()
    mult = C.c_int32()
    lib().orc_coarsest_dense(g.n, rp, col, w, seed, y, C.byref(lam), C.byref(mult))
    return y, float(lam.value), int(mult.value)


def pi(g, y0, tol: float = 1e-8, maxit: int = 100000, gval: float | None = None):
    rp, col, w = _csr_args(g)
    if gval is None:
        gval = gershgorin(g)
    y = np.zeros(g.n)
    margin = C.c_double()
    k = lib().orc_pi(g.n, rp, col, w, gval, np.ascontiguousarray(y0, dtype=np.float64), tol, maxit, y,
                     C.byref(margin))
    return y, int(k), float(margin.value)


def rq_residual(g, y):
    rp, col, w = _csr_args(g)
    rq = C.c_double()
    res = C.c_double()
    lib().orc_rq_residual(g.n, rp, col, w, np.ascontiguousarray(y, dtype=np.float64), C.byref(rq),
                          C.byref(res))
    return float(rq.value), float(res.value)


# ------------------------------------------------------------------ driver

@dataclasses.dataclass
class Level:
    n: int
    nnz: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray
    agg: np.ndarray | None
    g: float
    k: int
    margin: float


@dataclasses.dataclass
class Result:
    status: str
    levels: list
    lam: float
    residual: float
    y: np.ndarray
    coarse_lambda2: float
    coarse_mult: int
    collapsed: bool


def cmg(g, tol: float = 1e-8, coarsest_n: int = 25, dense_max: int = 128, seed: int = 14120565,
        max_iters: int = 100000, keep_levels: bool = True, fixed_k0: int = 0, fixed_beta: float = 2.0,
        coarsen: str = "hec") -> Result:
    """Full CMG (Algorithm 1) on the CPU oracle.  fixed_k0 > 0: Algorithm
    4's schedule k_j = ceil(fixed_k0 fixed_beta^j) steps per level instead
    of the stopping test; coarsen "hem": heavy edge matching instead of HEC."""
    L = lib()
    rp, col, w = _csr_args(g)
    r = L.orc_cmg_ex(g.n, int(rp[-1]), rp, col, w, tol, coarsest_n, dense_max, seed, max_iters,
                     int(fixed_k0), float(fixed_beta), {"hec": 0, "hem": 1}[coarsen])
    if not r:
        raise MemoryError
    try:
        st = STATUS[L.orc_res_status(r)]
        if st not in ("OK", "W_MAXIT"):
            return Result(st, [], float("nan"), float("nan"), np.zeros(0), float("nan"), 0, False)
        levels = []
        nl = L.orc_res_nlevels(r)
        for j in range(nl):
            n = L.orc_res_level_n(r, j)
            nz = L.orc_res_level_nnz(r, j)
            if keep_levels:
                lrp = np.zeros(n + 1, dtype=np.int32)
                lcol = np.zeros(nz, dtype=np.int32)
                lw = np.zeros(nz, dtype=np.float64)
                agg = np.zeros(n, dtype=np.int32) if j < nl - 1 else None
                L.orc_res_copy_level(r, j, lrp.ctypes.data, lcol.ctypes.data, lw.ctypes.data,
                                     agg.ctypes.data if agg is not None else None)
            else:
                lrp = lcol = lw = agg = None
            levels.append(Level(n, nz, lrp, lcol, lw, agg, L.orc_res_level_g(r, j), L.orc_res_level_k(r, j),
                                L.orc_res_level_margin(r, j)))
        y = np.zeros(g.n)
        L.orc_res_copy_y(r, y)
        return Result(st, levels, L.orc_res_lambda(r), L.orc_res_residual(r), y,
                      L.orc_res_coarse_lambda2(r), L.orc_res_coarse_mult(r), bool(L.orc_res_collapsed(r)))
    finally:
        L.orc_free(r)


@dataclasses.dataclass
class BlockResult:
    status: str
    k: list
    lams: np.ndarray
    residuals: np.ndarray
    coarse: np.ndarray
    X: np.ndarray  # n x p


def coarsest_block(g, p: int, seed: int = 14120565):
    rp, col, w = _csr_args(g)
    V = np.zeros(g.n * p)
    lams = np.zeros(p)
    st = lib().orc_coarsest_block(g.n, rp, col, w, seed, p, V, lams)
    if st != 0:
        raise ValueError(STATUS[st])
    return V.reshape(p, g.n).T.copy(), lams


def block_pi(g, V0, tol: float = 1e-8, maxit: int = 100000, steps: int = 0, gval: float | None = None):
    rp, col, w = _csr_args(g)
    if gval is None:
        gval = gershgorin(g)
    p = V0.shape[1]
    v0 = np.ascontiguousarray(V0.T, dtype=np.float64).reshape(-1)
    V = np.zeros(g.n * p)
    mu = C.c_double()
    k = lib().orc_block_pi(g.n, rp, col, w, gval, p, v0, tol, maxit, steps, V, C.byref(mu))
    return V.reshape(p, g.n).T.copy(), int(k), float(mu.value)


def cmg_block(g, p: int, tol: float = 1e-8, coarsest_n: int = 25, dense_max: int = 128,
              seed: int = 14120565, max_iters: int = 100000, fixed_k0: int = 0,
              fixed_beta: float = 2.0) -> BlockResult:
    """Several eigenpairs (Remark after Algorithm 4) on the oracle."""
    L = lib()
    rp, col, w = _csr_args(g)
    r = L.orc_cmg_block(g.n, int(rp[-1]), rp, col, w, tol, coarsest_n, dense_max, seed, max_iters,
                        int(fixed_k0), float(fixed_beta), int(p))
    if not r:
        raise MemoryError
    try:
        st = STATUS[L.orc_block_status(r)]
        nl = L.orc_block_nlevels(r)
        X = np.zeros(g.n * p)
        if st in ("OK", "W_MAXIT"):
            L.orc_block_copy_x(r, g.n, X)
        return BlockResult(st, [L.orc_block_k(r, j) for j in range(nl)],
                           np.array([L.orc_block_lambda(r, c) for c in range(p)]),
                           np.array([L.orc_block_residual(r, c) for c in range(p)]),
                           np.array([L.orc_block_coarse(r, c) for c in range(p)]),
                           X.reshape(p, g.n).T.copy())
    finally:
        L.orc_block_free(r)


def rsb(g, depth: int) -> np.ndarray:
    """Recursive spectral bisection into 2^depth parts on the oracle."""
    rp, col, w = _csr_args(g)
    part = np.zeros(g.n, dtype=np.int32)
    st = lib().orc_rsb(g.n, int(rp[-1]), rp, col, w, depth, part)
    if st != 0:
        raise ValueError(STATUS[st])
    return part


def components(g) -> np.ndarray:
    """comp[v] = smallest vertex of v's connected component."""
    rp, col, _ = _csr_args(g)
    comp = np.zeros(g.n, dtype=np.int32)
    lib().orc_components(g.n, rp, col, comp)
    return comp
