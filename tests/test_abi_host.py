"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/rihvr.h, its struct layouts match the
Python binding, and argument validation rejects bad input before any launch."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_1904_04884_amd import rihvr, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rihvr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ri_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not rihvr.LIB_PATH.exists():
        pytest.fail("librihvr.so is not built (run __graft_entry__.build())")
    return rihvr.lib()


def test_header_declares_the_binding_names():
    assert set(declared_functions()) == set(rihvr.EXPORTED)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", str(rihvr.LIB_PATH)], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ri_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_struct_layouts_match_header():
    """Compile a probe against the header with gcc and compare sizes / offsets."""
    probe = r"""
#include <stdio.h>
#include <stddef.h>
#include "rihvr.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("ri_geometry %zu\n", sizeof(ri_geometry));
  printf("ri_prox_params %zu\n", sizeof(ri_prox_params));
  printf("ri_solve_params %zu\n", sizeof(ri_solve_params));
  printf("ri_solve_report %zu\n", sizeof(ri_solve_report));
  printf("ri_tuning %zu\n", sizeof(ri_tuning));
  printf("ri_autotune_report %zu\n", sizeof(ri_autotune_report));
  F(ri_geometry, pixel_um) F(ri_geometry, flags)
  F(ri_prox_params, inner_iters) F(ri_prox_params, nonneg)
  F(ri_solve_params, gap_tol) F(ri_solve_params, init) F(ri_solve_params, flags) F(ri_solve_params, nonneg)
  F(ri_solve_params, x0_scale)
  F(ri_solve_report, objective) F(ri_solve_report, phase_ms) F(ri_solve_report, phase_launches)
  F(ri_tuning, tv_blocks) F(ri_tuning, col_blocks)
  F(ri_autotune_report, from_cache) F(ri_autotune_report, candidates) F(ri_autotune_report, default_ms)
  F(ri_autotune_report, tune_ms)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(src, "w").write(probe)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.rsplit(" ", 1) for l in lines if l.strip())
    ctypes_side = {
        "ri_geometry": C.sizeof(rihvr.ri_geometry),
        "ri_prox_params": C.sizeof(rihvr.ri_prox_params),
        "ri_solve_params": C.sizeof(rihvr.ri_solve_params),
        "ri_solve_report": C.sizeof(rihvr.ri_solve_report),
        "ri_tuning": C.sizeof(rihvr.ri_tuning),
        "ri_autotune_report": C.sizeof(rihvr.ri_autotune_report),
    }
    for k, v in ctypes_side.items():
        assert int(got[k]) == v, k
    for key, val in got.items():
        if "." in key:
            struct, field = key.split(".")
            assert getattr(getattr(rihvr, struct), field).offset == int(val), key


def test_status_strings(lib):
    for s in range(8):
        assert rihvr.ri_status_string(s)
    assert rihvr.ri_status_string(0) == "ok"


@pytest.mark.parametrize("nx,ny,nz", [(1000, 1024, 4), (1024, 1000, 4), (8, 16, 1), (4096, 64, 1),
                                      (16, 16, 0), (18, 16, 1)])
def test_plan_rejects_unsupported_geometry(lib, nx, ny, nz):
    g = scenes.geometry_c1().with_(nx=nx, ny=ny, nz=nz)
    h = C.c_void_p()
    st = lib.ri_plan_create(C.byref(rihvr.geometry_struct(g)), rihvr.RI_F32, C.byref(h))
    assert st in (rihvr.RI_ERR_UNSUPPORTED_SIZE, rihvr.RI_ERR_INVALID_ARG)
    assert h.value is None
    assert rihvr.ri_last_error()


def test_plan_rejects_evanescent_and_bad_optics(lib):
    for kw in ({"pixel_um": 0.4}, {"wavelength_um": -1.0}, {"pixel_um": 0.0}):
        g = scenes.geometry_c1().with_(**kw)
        h = C.c_void_p()
        assert lib.ri_plan_create(C.byref(rihvr.geometry_struct(g)), rihvr.RI_F32, C.byref(h)) == rihvr.RI_ERR_INVALID_ARG


def test_header_signatures_of_the_boundary():
    """The entry points have the boundary's signatures: plain pointers and
    sizes, the element type chosen per plan.  A C probe assigns each to a
    pointer of the expected type; gcc rejects any mismatch."""
    probe = r"""
#include "rihvr.h"
ri_status (*pc)(const ri_geometry*, ri_dtype, ri_plan**) = ri_plan_create;
ri_status (*pw)(const ri_plan*, size_t*) = ri_workspace_size;
ri_status (*pwo)(const ri_plan*, ri_op, size_t*) = ri_workspace_size_op;
ri_status (*pf)(ri_plan*, const void*, void*, void*, size_t, void*) = ri_forward;
ri_status (*pa)(ri_plan*, const void*, void*, void*, size_t, void*) = ri_adjoint;
ri_status (*pp)(ri_plan*, const ri_prox_params*, double, const void*, void*, void*, size_t, void*) =
    ri_prox_fused_lasso;
ri_status (*ps)(ri_plan*, const ri_solve_params*, const void*, void*, void*, size_t, void*, ri_solve_report*) =
    ri_solve;
ri_status (*pb)(int32_t, ri_plan* const*, const ri_solve_params*, const void* const*, void* const*, void*, size_t,
                void*, ri_solve_report*) = ri_solve_batched;
const char* (*pe)(void) = ri_last_error;
int main(void) { return (int)RI_F64 - 1 + (int)RI_F32; }
"""
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "sig.c")
        open(src, "w").write(probe)
        r = subprocess.run(["gcc", "-Werror", "-Wincompatible-pointer-types", "-c", "-I",
                            os.path.join(ROOT, "include"), src, "-o", os.path.join(d, "sig.o")],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_plan_rejects_unknown_dtype(lib):
    g = scenes.geometry_c1().with_(nx=64, ny=64, nz=4)
    h = C.c_void_p()
    assert lib.ri_plan_create(C.byref(rihvr.geometry_struct(g)), 7, C.byref(h)) == rihvr.RI_ERR_INVALID_ARG
    assert h.value is None


def test_null_arguments_rejected(lib):
    assert lib.ri_plan_create(None, rihvr.RI_F32, None) == rihvr.RI_ERR_INVALID_ARG
    n = C.c_size_t()
    assert lib.ri_workspace_size(None, C.byref(n)) == rihvr.RI_ERR_INVALID_ARG
    assert lib.ri_workspace_size_op(None, 0, C.byref(n)) == rihvr.RI_ERR_INVALID_ARG
    assert lib.ri_forward(None, None, None, None, 0, None) == rihvr.RI_ERR_INVALID_ARG
    assert lib.ri_adjoint(None, None, None, None, 0, None) == rihvr.RI_ERR_INVALID_ARG
    p = rihvr.ri_prox_params(0.1, 0.1, 3, 1)
    assert lib.ri_prox_fused_lasso(None, C.byref(p), 1.0, None, None, None, 0, None) == rihvr.RI_ERR_INVALID_ARG
    sp = rihvr.ri_solve_params()
    assert lib.ri_solve(None, C.byref(sp), None, None, None, 0, None, None) == rihvr.RI_ERR_INVALID_ARG
    assert lib.ri_plan_destroy(None) == rihvr.RI_ERR_INVALID_ARG
    t = rihvr.ri_tuning(3, 1536, 512)
    assert lib.ri_plan_get_tuning(None, C.byref(t)) == rihvr.RI_ERR_INVALID_ARG
    assert lib.ri_plan_set_tuning(None, C.byref(t)) == rihvr.RI_ERR_INVALID_ARG
    assert lib.ri_plan_autotune(None, 10, None, None, 0, None, None) == rihvr.RI_ERR_INVALID_ARG
    assert lib.ri_workspace_size_op(None, rihvr.RI_OP_AUTOTUNE, C.byref(n)) == rihvr.RI_ERR_INVALID_ARG
    assert rihvr.ri_solve_batched(0, [], [], [], [], None, 0, None) == rihvr.RI_OK
    assert lib.ri_solve_batched(-1, None, None, None, None, None, 0, None, None) == rihvr.RI_ERR_INVALID_ARG


def test_scenes_are_seeded_and_in_bounds():
    a = scenes.scene_c1(seed=3)
    b = scenes.scene_c1(seed=3)
    c = scenes.scene_c1(seed=4)
    assert np.array_equal(a.idx, b.idx) and np.array_equal(a.noise, b.noise)
    assert not np.array_equal(a.idx, c.idx)
    g = a.geometry
    assert a.idx.min() >= 0 and np.all(a.idx.max(axis=0) < np.array(g.shape))
    assert len(a.centers) == 50
    d = scenes.disk_particles(g, 20, np.random.default_rng(0))
    assert d[1].max() <= 1.0 and d[1].min() > 0.0
