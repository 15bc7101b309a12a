"""Thin Python binding of libcmg (include/cmg.h).

Argument marshalling only: every step of the method runs in the HIP
kernels of ``libcmg.so``.  Functions keep the C names.  Arrays may be numpy
arrays (host memory) or torch tensors (device memory on the current GPU);
torch is used only for device memory and streams.

Loading fails loudly if the HIP library has not been built: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_PKG, "libcmg.so")

CMG_OK, CMG_E_ARG, CMG_E_GRAPH, CMG_E_ISOLATED, CMG_E_OOM, CMG_E_DEVICE, CMG_W_MAXIT = range(7)
CMG_FP64, CMG_MIXED = 0, 1
CMG_MEM_HOST, CMG_MEM_DEVICE = 0, 1
CMG_VAL_F64, CMG_VAL_F32 = 0, 1

# functions declared in include/cmg.h
EXPORTS = ["cmg_options_default", "cmg_setup", "cmg_fiedler", "cmg_fiedler_batch", "cmg_level_info",
           "cmg_level_copy", "cmg_set_stream", "cmg_footprint", "cmg_free", "cmg_status_string",
           "cmg_last_error", "cmg_hash_probe", "cmg_fiedler_noalloc", "cmg_fiedler_block", "cmg_bisect"]

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class cmg_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class cmg_options(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("tol", C.c_double),
        ("coarsest_n", C.c_int32),
        ("dense_max", C.c_int32),
        ("seed", C.c_uint64),
        ("precision", C.c_int32),
        ("fp64_final_sweeps", C.c_int32),
        ("max_iters_per_level", C.c_int32),
        ("validate_full", C.c_int32),
        ("stream", C.c_void_p),
        ("allocator", C.POINTER(cmg_allocator)),
        ("block_rows", C.c_int32),
        ("mixed_min_nnz", C.c_int64),
        ("spmv_variant", C.c_int32),
        ("autotune", C.c_int32),
        ("block_regs", C.c_int32),
        ("grid_stage", C.c_int32),
        ("step_mode", C.c_int32),
        ("fixed_k0", C.c_int32),
        ("fixed_beta", C.c_double),
        ("graph", C.c_int32),
        ("coarsen", C.c_int32),
        ("galerkin", C.c_int32),
        ("test_abort_level", C.c_int32),
        ("weight_storage", C.c_int32),
    ]


class cmg_level_stats(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("nnz", C.c_int64),
        ("g", C.c_double),
        ("wmax", C.c_double),
        ("k", C.c_int32),
        ("margin", C.c_double),
        ("fp32", C.c_int32),
        ("in_block", C.c_int32),
        ("variant", C.c_int32),
        ("lanes", C.c_int32),
        ("grid", C.c_int32),
        ("pi_ms", C.c_double),
        ("bytes_per_iter", C.c_double),
        ("block_waves", C.c_int32),
        ("block_regs", C.c_int32),
        ("step", C.c_int32),
        ("weights", C.c_int32),
        ("block_slots", C.c_int32),
    ]


class cmg_stats(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("nlevels", C.c_int32),
        ("collapsed", C.c_int32),
        ("hec_rounds", C.c_int32),
        ("lambda_", C.c_double),
        ("residual", C.c_double),
        ("coarse_lambda2", C.c_double),
        ("coarse_mult", C.c_int32),
        ("setup_ms", C.c_double),
        ("fiedler_ms", C.c_double),
        ("finest_pi_ms", C.c_double),
        ("finest_k", C.c_int32),
        ("finest_bytes", C.c_double),
        ("status", C.c_int32),
        ("fallback", C.c_int32),
    ]


_lib = None


def lib():
    """Load libcmg.so (raises if it is missing: no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"libcmg.so not built ({LIBPATH}); run python -m paper_1412_0565_amd.build")
        L = C.CDLL(LIBPATH)
        L.cmg_options_default.argtypes = [C.POINTER(cmg_options)]
        L.cmg_options_default.restype = None
        L.cmg_setup.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                C.POINTER(cmg_options), C.POINTER(C.c_void_p)]
        L.cmg_setup.restype = C.c_int
        L.cmg_fiedler.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_int, C.POINTER(cmg_stats)]
        L.cmg_fiedler.restype = C.c_int
        L.cmg_fiedler_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_double),
                                        C.POINTER(C.c_void_p), C.c_int, C.POINTER(cmg_stats)]
        L.cmg_fiedler_batch.restype = C.c_int
        L.cmg_level_info.argtypes = [C.c_void_p, C.POINTER(cmg_level_stats), C.c_int32, C.POINTER(C.c_int32)]
        L.cmg_level_info.restype = C.c_int
        L.cmg_level_copy.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.cmg_level_copy.restype = C.c_int
        L.cmg_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        L.cmg_set_stream.restype = C.c_int
        L.cmg_footprint.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.cmg_footprint.restype = C.c_int
        L.cmg_free.argtypes = [C.c_void_p]
        L.cmg_free.restype = None
        L.cmg_status_string.argtypes = [C.c_int]
        L.cmg_status_string.restype = C.c_char_p
        L.cmg_last_error.argtypes = []
        L.cmg_last_error.restype = C.c_char_p
        L.cmg_hash_probe.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_void_p]
        L.cmg_hash_probe.restype = C.c_int
        L.cmg_fiedler_noalloc.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                          C.c_int, C.POINTER(cmg_options), C.POINTER(C.c_double), C.c_void_p,
                                          C.POINTER(cmg_stats)]
        L.cmg_fiedler_noalloc.restype = C.c_int
        L.cmg_fiedler_block.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                        C.c_void_p]
        L.cmg_fiedler_block.restype = C.c_int
        L.cmg_bisect.argtypes = [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                 C.POINTER(cmg_options), C.c_int32, C.c_void_p, C.POINTER(C.c_double)]
        L.cmg_bisect.restype = C.c_int
        _lib = L
    return _lib


class CmgError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        detail = cmg_last_error()
        super().__init__(f"{where}: {cmg_status_string(status)}" + (f" [{detail}]" if detail else ""))


def _check(st: int, where: str) -> int:
    if st not in (CMG_OK, CMG_W_MAXIT):
        raise CmgError(st, where)
    return st


def cmg_status_string(status: int) -> str:
    return lib().cmg_status_string(status).decode()


def cmg_last_error() -> str:
    return lib().cmg_last_error().decode()


def cmg_options_default(**overrides) -> cmg_options:
    o = cmg_options()
    lib().cmg_options_default(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def _ptr(a):
    """(pointer, memspace) of a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C contiguous")
        return a.ctypes.data, CMG_MEM_HOST
    import torch

    if isinstance(a, torch.Tensor):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), (CMG_MEM_DEVICE if a.is_cuda else CMG_MEM_HOST)
    raise TypeError(type(a))


# ------------------------------------------------------------ torch memory

_torch_alloc_keep = []


def torch_allocator() -> cmg_allocator:
    """cmg_allocator backed by torch's caching allocator on the current device."""
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream or 0))
        except Exception:
            return None

    def _free(p, stream, user):
        torch.cuda.caching_allocator_delete(int(p))

    a = cmg_allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)
    _torch_alloc_keep.append(a)
    return a


# ------------------------------------------------------------------- ABI

def cmg_setup(n: int, row_ptr, col, w, opt: cmg_options | None = None) -> int:
    """Returns the handle (int).  row_ptr/col int32, w float64 or float32,
    all host (numpy) or all device (torch) arrays."""
    prp, where = _ptr(row_ptr)
    pcol, w2 = _ptr(col)
    pw, w3 = _ptr(w)
    if not (where == w2 == w3):
        raise ValueError("row_ptr, col and w must share one memory space")
    if str(row_ptr.dtype).split(".")[-1] != "int32" or str(col.dtype).split(".")[-1] != "int32":
        raise TypeError("row_ptr and col must be int32")
    wt = str(w.dtype).split(".")[-1]
    if wt not in ("float64", "float32"):
        raise TypeError("w must be float64 or float32")
    wtype = CMG_VAL_F32 if wt == "float32" else CMG_VAL_F64
    nnz = int(col.shape[0])
    h = C.c_void_p()
    st = lib().cmg_setup(int(n), nnz, prp, pcol, pw, wtype, where,
                         C.byref(opt) if opt is not None else None, C.byref(h))
    _check(st, "cmg_setup")
    return h.value


def cmg_fiedler(h: int, x=None, stats: cmg_stats | None = None):
    """Runs the solve; returns (lambda, status).  x: float64 output array
    (numpy host or torch device) of n entries, or None."""
    lam = C.c_double()
    px, where = (None, CMG_MEM_HOST) if x is None else _ptr(x)
    st = lib().cmg_fiedler(h, C.byref(lam), px, where, C.byref(stats) if stats is not None else None)
    _check(st, "cmg_fiedler")
    return lam.value, st


def cmg_fiedler_batch(hs, xs=None, stats=None):
    n = len(hs)
    harr = (C.c_void_p * n)(*hs)
    lams = (C.c_double * n)()
    where = CMG_MEM_HOST
    xarr = None
    if xs is not None:
        ptrs = []
        for x in xs:
            p, where = _ptr(x)
            ptrs.append(p)
        xarr = (C.c_void_p * n)(*ptrs)
    sarr = None
    if stats is not None:
        sarr = (cmg_stats * n)()
    st = lib().cmg_fiedler_batch(harr, n, lams, xarr, where, sarr)
    _check(st, "cmg_fiedler_batch")
    if stats is not None:
        stats.extend(list(sarr))
    return list(lams), st


def cmg_fiedler_block(h: int, p: int, X=None):
    """Several eigenpairs on the handle's hierarchy.  X: float64 n x p
    output, column-major (numpy array of shape (p, n), or a torch tensor
    of p n entries), or None.  Returns (lambdas, residuals, level_steps,
    status)."""
    lams = np.zeros(p)
    res = np.zeros(p)
    nl = C.c_int32()
    _check(lib().cmg_level_info(h, None, 0, C.byref(nl)), "cmg_level_info")
    steps = np.zeros(nl.value, dtype=np.int32)
    px, where = (None, CMG_MEM_HOST) if X is None else _ptr(X)
    st = lib().cmg_fiedler_block(h, int(p), lams.ctypes.data, px, where, res.ctypes.data, steps.ctypes.data)
    _check(st, "cmg_fiedler_block")
    return lams, res, [int(k) for k in steps], st


def cmg_bisect(n: int, row_ptr, col, w, depth: int, part=None, opt: cmg_options | None = None):
    """Recursive spectral bisection into 2^depth parts.  Arrays as
    cmg_setup; part: int32 output of n entries in the same memory space
    (a new numpy array if None).  Returns (part, cut)."""
    prp, where = _ptr(row_ptr)
    pcol, _ = _ptr(col)
    pw, _ = _ptr(w)
    if part is None:
        part = np.zeros(int(n), dtype=np.int32)
    pp, _ = _ptr(part)
    wtype = CMG_VAL_F32 if str(w.dtype).split(".")[-1] == "float32" else CMG_VAL_F64
    cut = C.c_double()
    st = lib().cmg_bisect(int(n), int(col.shape[0]), prp, pcol, pw, wtype, where,
                          C.byref(opt) if opt is not None else None, int(depth), pp, C.byref(cut))
    _check(st, "cmg_bisect")
    return part, cut.value


def cmg_level_info(h: int):
    nl = C.c_int32()
    _check(lib().cmg_level_info(h, None, 0, C.byref(nl)), "cmg_level_info")
    arr = (cmg_level_stats * nl.value)()
    _check(lib().cmg_level_info(h, arr, nl.value, C.byref(nl)), "cmg_level_info")
    return list(arr)


def cmg_level_copy(h: int, level: int, n: int, nnz: int, with_agg: bool = True):
    rp = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(nnz, dtype=np.int32)
    w = np.zeros(nnz, dtype=np.float64)
    agg = np.zeros(n, dtype=np.int32) if with_agg else None
    _check(lib().cmg_level_copy(h, level, rp.ctypes.data, col.ctypes.data, w.ctypes.data,
                                agg.ctypes.data if agg is not None else None), "cmg_level_copy")
    return rp, col, w, agg


def cmg_set_stream(h: int, stream) -> None:
    """stream: a torch.cuda.Stream, a raw hipStream_t (int), or None."""
    raw = getattr(stream, "cuda_stream", stream)
    _check(lib().cmg_set_stream(h, C.c_void_p(raw) if raw else None), "cmg_set_stream")


def cmg_footprint(h: int) -> int:
    b = C.c_size_t()
    _check(lib().cmg_footprint(h, C.byref(b)), "cmg_footprint")
    return b.value


def cmg_free(h: int) -> None:
    lib().cmg_free(h)


def cmg_fiedler_noalloc(n: int, row_ptr, col, w, x, opt: cmg_options | None = None,
                        stats: cmg_stats | None = None):
    """Setup + solve + free in one call that allocates no device memory
    (static scratch).  Arrays as cmg_setup; x: float64 output of n entries
    in the same memory space.  Returns (lambda, status)."""
    prp, where = _ptr(row_ptr)
    pcol, w2 = _ptr(col)
    pw, w3 = _ptr(w)
    px, w4 = _ptr(x)
    if not (where == w2 == w3 == w4):
        raise ValueError("row_ptr, col, w and x must share one memory space")
    wtype = CMG_VAL_F32 if str(w.dtype).split(".")[-1] == "float32" else CMG_VAL_F64
    lam = C.c_double()
    st = lib().cmg_fiedler_noalloc(int(n), int(col.shape[0]), prp, pcol, pw, wtype, where,
                                   C.byref(opt) if opt is not None else None, C.byref(lam), px,
                                   C.byref(stats) if stats is not None else None)
    _check(st, "cmg_fiedler_noalloc")
    return lam.value, st


def cmg_hash_probe(seed: int, level: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _check(lib().cmg_hash_probe(seed, level, count, out.ctypes.data), "cmg_hash_probe")
    return out


# ------------------------------------------------------------ convenience

class Fiedler:
    """Owns one hierarchy: ``Fiedler(graph_arrays...).solve()``.

    A context manager wrapper over cmg_setup / cmg_fiedler / cmg_free.
    """

    def __init__(self, n, row_ptr, col, w, **opts):
        self.n = int(n)
        self.opt = cmg_options_default(**opts)
        self.handle = cmg_setup(n, row_ptr, col, w, self.opt)

    def solve(self, x=None):
        st = cmg_stats()
        st.struct_size = C.sizeof(cmg_stats)
        if x is None:
            x = np.zeros(self.n)
        lam, status = cmg_fiedler(self.handle, x, st)
        return lam, x, st

    def solve_block(self, p: int):
        """p eigenpairs: (lambdas, X of shape (n, p), residuals, level_steps)."""
        X = np.zeros((p, self.n))
        lams, res, steps, _ = cmg_fiedler_block(self.handle, p, X)
        return lams, X.T.copy(), res, steps

    def levels(self):
        return cmg_level_info(self.handle)

    def level_arrays(self, j):
        info = self.levels()
        last = j == len(info) - 1
        return cmg_level_copy(self.handle, j, info[j].n, int(info[j].nnz), with_agg=not last)

    def footprint(self):
        return cmg_footprint(self.handle)

    def close(self):
        if self.handle:
            cmg_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
