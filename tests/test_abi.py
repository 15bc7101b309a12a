"""C-ABI checks that need no GPU: the library loads, exports every function
include/cmg.h declares, its structs match the binding's layout, and the
pure-host paths (defaults, status strings, argument errors) behave."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmg.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\*]+\s+\**(cmg_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def cmg():
    from paper_1412_0565_amd import cmg as M

    if not os.path.exists(M.LIBPATH):
        pytest.fail("libcmg.so is not built (python -m paper_1412_0565_amd.build)")
    return M


def test_exports_every_declared_symbol(cmg):
    decl = _declared_functions()
    assert len(decl) >= 10
    lib = C.CDLL(cmg.LIBPATH)
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(cmg.EXPORTS) == decl


def test_nm_shows_c_linkage(cmg):
    out = subprocess.run(["nm", "-D", "--defined-only", cmg.LIBPATH], capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for name in _declared_functions():
        assert name in syms, name  # unmangled: extern "C"


def test_struct_layout_matches_header(cmg, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "cmg.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("cmg_options %zu\n", sizeof(cmg_options));
  printf("cmg_stats %zu\n", sizeof(cmg_stats));
  printf("cmg_level_stats %zu\n", sizeof(cmg_level_stats));
  printf("cmg_allocator %zu\n", sizeof(cmg_allocator));
  F(cmg_options, tol) F(cmg_options, seed) F(cmg_options, stream) F(cmg_options, allocator)
  F(cmg_options, block_rows) F(cmg_options, mixed_min_nnz) F(cmg_options, spmv_variant)
  F(cmg_options, grid_stage) F(cmg_options, step_mode) F(cmg_level_stats, step)
  F(cmg_options, fixed_k0) F(cmg_options, fixed_beta) F(cmg_options, graph) F(cmg_options, coarsen) F(cmg_options, galerkin)
  F(cmg_options, test_abort_level) F(cmg_options, weight_storage) F(cmg_stats, fallback) F(cmg_level_stats, weights)
  F(cmg_stats, lambda) F(cmg_stats, residual) F(cmg_stats, finest_bytes) F(cmg_stats, status)
  F(cmg_level_stats, nnz) F(cmg_level_stats, pi_ms) F(cmg_level_stats, bytes_per_iter) F(cmg_level_stats, block_slots)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(got["cmg_options"]) == C.sizeof(cmg.cmg_options)
    assert int(got["cmg_stats"]) == C.sizeof(cmg.cmg_stats)
    assert int(got["cmg_level_stats"]) == C.sizeof(cmg.cmg_level_stats)
    assert int(got["cmg_allocator"]) == C.sizeof(cmg.cmg_allocator)
    pyname = {"lambda": "lambda_"}
    for k, v in got.items():
        if "." in k:
            t, m = k.split(".")
            cls = getattr(cmg, t)
            assert getattr(cls, pyname.get(m, m)).offset == int(v), k


def test_options_default(cmg):
    o = cmg.cmg_options_default()
    assert o.struct_size == C.sizeof(cmg.cmg_options)
    assert o.tol == 1e-8 and o.coarsest_n == 25 and o.dense_max == 128
    assert o.seed == 14120565 and o.precision == cmg.CMG_FP64
    assert o.fp64_final_sweeps == 1 and o.max_iters_per_level == 100000


def test_status_strings(cmg):
    for s in range(7):
        assert cmg.cmg_status_string(s).startswith("CMG_")
    assert "unknown" in cmg.cmg_status_string(99)


def test_argument_errors_are_host_side(cmg):
    L = cmg.lib()
    h = C.c_void_p()
    one = (C.c_int32 * 2)(0, 0)
    # NULL out, n < 2, NULL arrays, bad enums: rejected before any HIP call
    assert L.cmg_setup(4, 2, one, one, one, 0, 0, None, None) == cmg.CMG_E_ARG
    assert L.cmg_setup(1, 2, one, one, one, 0, 0, None, C.byref(h)) == cmg.CMG_E_ARG
    assert h.value is None
    assert L.cmg_setup(4, 2, None, one, one, 0, 0, None, C.byref(h)) == cmg.CMG_E_ARG
    assert L.cmg_setup(4, 2, one, one, one, 7, 0, None, C.byref(h)) == cmg.CMG_E_ARG
    assert L.cmg_setup(4, 2, one, one, one, 0, 9, None, C.byref(h)) == cmg.CMG_E_ARG
    bad = cmg.cmg_options_default(dense_max=500)
    assert L.cmg_setup(4, 2, one, one, one, 0, 0, C.byref(bad), C.byref(h)) == cmg.CMG_E_ARG
    bad = cmg.cmg_options_default(tol=float("nan"))
    assert L.cmg_setup(4, 2, one, one, one, 0, 0, C.byref(bad), C.byref(h)) == cmg.CMG_E_ARG
    assert L.cmg_fiedler(None, None, None, 0, None) == cmg.CMG_E_ARG
    assert L.cmg_level_info(None, None, 0, None) == cmg.CMG_E_ARG
    L.cmg_free(None)  # no-op


def test_binding_has_no_cpu_fallback(cmg, monkeypatch):
    monkeypatch.setattr(cmg, "_lib", None)
    monkeypatch.setattr(cmg, "LIBPATH", "/nonexistent/libcmg.so")
    with pytest.raises(RuntimeError):
        cmg.lib()


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1412_0565_amd")
    bad = re.compile(r"^\s*(import\s+oracle|from\s+oracle)|liboracle|cmg_oracle|\borc_\w+\(", re.M)
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert not bad.search(txt), f
