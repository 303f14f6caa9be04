"""The C ABI on the host: the library loads, exports every declared symbol,
and validates arguments before touching the device (runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import grid as ogrid
from paper_2502_06296_amd import _native as N
from paper_2502_06296_amd import solver

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "pf_channel.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_exports():
    assert _declared_functions() == sorted(N.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = N.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    assert L.pf_abi_version() == 3


@pytest.mark.parametrize("bc", [0, 1, 2])
@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_host_z_rows_match_oracle(bc, beta):
    nz = 37
    a, g, e = solver.zop_rows(nz, bc, lz=2.0, beta=beta)
    zf = synth.tanh_faces(nz, 2.0, beta)
    ra, rg, re_ = ogrid.zop(zf, bc)
    for x, y in ((a, ra), (g, rg), (e, re_)):
        np.testing.assert_allclose(x, y, rtol=1e-13, atol=0)


def test_host_faces_match_generator():
    for beta in (0.0, 1.0, 1.5, 2.0):
        zf = solver.grid_faces(64, 64, 96, beta=beta)
        np.testing.assert_allclose(zf, synth.tanh_faces(96, 2.0, beta), rtol=1e-15, atol=1e-15)
    user = np.cumsum(np.r_[0.0, np.linspace(1, 2, 10)])
    np.testing.assert_array_equal(solver.grid_faces(64, 64, 10, zf=user), user)


def _plan_status(nx, ny, nz, prec=0, nref=1, zf=None, beta=1.5):
    g, keep = N.make_grid(nx, ny, nz, 2 * np.pi, np.pi, 2.0, beta, zf)
    h = C.c_void_p()
    ws = C.c_size_t(0)
    return N.lib().poisson_plan(C.byref(h), C.byref(g), prec, nref, None, C.byref(ws))


@pytest.mark.parametrize("args,code", [
    ((100, 64, 64), N.PF_ERR_UNSUPPORTED),   # 100 = 4*25 not built
    ((64, 80, 64), N.PF_ERR_UNSUPPORTED),
    ((64, 64, 3), N.PF_ERR_ARG),              # nz too small
    ((64, 64, 2048), N.PF_ERR_UNSUPPORTED),   # nz too large
    ((4096, 64, 64), N.PF_ERR_UNSUPPORTED),
    ((64, 3000, 64), N.PF_ERR_UNSUPPORTED),  # 2^3 3 5^3: a length not in the built list
])
def test_plan_rejects_bad_grids_before_any_device_call(args, code):
    assert _plan_status(*args) == code
    assert N.lib().pf_last_error()


def test_plan_validates_the_y_boundary_before_any_device_call():
    for ybc, code in ((4, N.PF_ERR_ARG), (-1, N.PF_ERR_ARG)):
        g, keep = N.make_grid(64, 64, 64, 2 * np.pi, np.pi, 2.0, 1.5, None, ybc)
        h, ws = C.c_void_p(), C.c_size_t(0)
        assert N.lib().poisson_plan(C.byref(h), C.byref(g), 0, 1, None, C.byref(ws)) == code
        assert b"ybc" in N.lib().pf_last_error()
    g, keep = N.make_grid(64, 64, 64, 2 * np.pi, np.pi, 2.0, 1.5, None, 4)
    h, ws = C.c_void_p(), C.c_size_t(0)
    assert N.lib().helmholtz3d_plan(C.byref(h), C.byref(g), 1, 1e-3, 0, 1, None, C.byref(ws)) == \
        N.PF_ERR_ARG


def test_y_faces_are_for_the_helmholtz_and_need_twice_the_rows_built():
    # a field on the y faces (ybc 3): the Poisson plan refuses it; the 3-D
    # Helmholtz takes one transform of 2 ny points, so ny = 100 (200 points)
    # and ny = 2048 (4096) are not built
    g, keep = N.make_grid(64, 32, 16, 2 * np.pi, np.pi, 2.0, 1.5, None, 3)
    h, ws = C.c_void_p(), C.c_size_t(0)
    assert N.lib().poisson_plan(C.byref(h), C.byref(g), 0, 1, None, C.byref(ws)) == N.PF_ERR_UNSUPPORTED
    assert b"helmholtz3d_plan only" in N.lib().pf_last_error()
    for ny in (100, 2048):
        g, keep = N.make_grid(64, ny, 16, 2 * np.pi, np.pi, 2.0, 1.5, None, 3)
        assert N.lib().helmholtz3d_plan(C.byref(h), C.byref(g), 1, 1e-3, 0, 1, None, C.byref(ws)) == \
            N.PF_ERR_UNSUPPORTED
        assert b"faces" in N.lib().pf_last_error()
    # the same along x (xbc 3)
    g, keep = N.make_grid(32, 64, 16, 2 * np.pi, np.pi, 2.0, 1.5, None, 0, 3)
    assert N.lib().poisson_plan(C.byref(h), C.byref(g), 0, 1, None, C.byref(ws)) == N.PF_ERR_UNSUPPORTED
    assert b"helmholtz3d_plan only" in N.lib().pf_last_error()
    for nx in (100, 2048):
        g, keep = N.make_grid(nx, 64, 16, 2 * np.pi, np.pi, 2.0, 1.5, None, 0, 3)
        assert N.lib().helmholtz3d_plan(C.byref(h), C.byref(g), 1, 1e-3, 0, 1, None, C.byref(ws)) == \
            N.PF_ERR_UNSUPPORTED
        assert b"faces" in N.lib().pf_last_error()
    g, keep = N.make_grid(64, 64, 16, 2 * np.pi, np.pi, 2.0, 1.5, None, 0, 4)
    assert N.lib().helmholtz3d_plan(C.byref(h), C.byref(g), 1, 1e-3, 0, 1, None, C.byref(ws)) == N.PF_ERR_ARG
    # 48 faces along x: a float32 y workgroup of 96-point columns takes 32 x slots
    g, keep = N.make_grid(48, 96, 16, 2 * np.pi, np.pi, 2.0, 1.5, None, 0, 3)
    assert N.lib().helmholtz3d_plan(C.byref(h), C.byref(g), 1, 1e-3, 2, 1, None, C.byref(ws)) == \
        N.PF_ERR_UNSUPPORTED
    assert b"multiple of 32" in N.lib().pf_last_error()


def test_plan_rejects_bad_precision_and_refinement():
    assert _plan_status(64, 64, 64, prec=7) == N.PF_ERR_ARG
    assert _plan_status(64, 64, 64, prec=2, nref=3) == N.PF_ERR_UNSUPPORTED


def test_plan_rejects_non_monotone_faces():
    zf = np.linspace(0, 2, 17)
    zf[5] = zf[4]
    assert _plan_status(64, 64, 16, zf=zf) == N.PF_ERR_ARG


def test_null_arguments():
    L = N.lib()
    assert L.poisson_solve(None, None, None) == N.PF_ERR_ARG
    assert L.poisson_project(None, None, None, None, None, None, 1.0, 0.0) == N.PF_ERR_ARG
    assert L.poisson_set_status(None, None, 1e-10) == N.PF_ERR_ARG
    assert L.pcr_apply(None, None, 64, 64) == N.PF_ERR_ARG
    assert L.poisson_set_workspace(None, None, 0) == N.PF_ERR_ARG
    assert L.pf_graph_begin(None) == N.PF_ERR_ARG
    assert L.pf_copy_kernel(None, None, 16, None) == N.PF_ERR_ARG
    assert L.poisson_destroy(None) == N.PF_OK


def test_helmholtz3d_plan_validates_before_any_device_call():
    L = N.lib()
    g, keep = N.make_grid(64, 64, 16, 2 * np.pi, np.pi, 2.0, 1.5, None)
    h = C.c_void_p()
    ws = C.c_size_t(0)
    for bc, s in ((N.PF_BC_NEUMANN, 0.1), (7, 0.1), (N.PF_BC_DIRICHLET_CENTRE, 0.0),
                  (N.PF_BC_DIRICHLET_FACE, -1.0), (N.PF_BC_DIRICHLET_FACE, float("inf"))):
        assert L.helmholtz3d_plan(C.byref(h), C.byref(g), bc, s, 0, 1, None, C.byref(ws)) == N.PF_ERR_ARG
        assert L.pf_last_error()
    assert L.helmholtz3d_solve(None, None, None) == N.PF_ERR_ARG
    assert L.helmholtz3d_update(None, 1.0) == N.PF_ERR_ARG


def test_task_batch_validates_before_any_device_call():
    L = N.lib()
    tasks = (N.PfTask * 2)()
    assert L.pf_run_batched(0, tasks, 4, None) == N.PF_OK          # nothing to do
    assert L.pf_run_batched(-1, tasks, 4, None) == N.PF_ERR_ARG
    assert L.pf_run_batched(1, None, 4, None) == N.PF_ERR_ARG
    assert L.pf_run_batched(1, tasks, 0, None) == N.PF_ERR_ARG     # lanes 1..8
    assert L.pf_run_batched(1, tasks, 9, None) == N.PF_ERR_ARG
    assert L.pf_run_batched(1, tasks, 4, None) == N.PF_ERR_ARG     # empty task
    tasks[0].ncomp = 5
    assert L.pf_run_batched(1, tasks, 4, None) == N.PF_ERR_ARG
    tasks[0].ncomp = 1                                              # NULL plan
    assert L.pf_run_batched(1, tasks, 4, None) == N.PF_ERR_ARG
    assert L.pf_last_error()


def test_pcr_prepare_rejects_bad_rows():
    L = N.lib()
    pd = C.POINTER(C.c_double)
    a = np.zeros(8); g = np.ones(8); e = np.zeros(8)
    h = C.c_void_p()
    # gamma[n-1] must be zero
    assert L.pcr_prepare(C.byref(h), 8, a.ctypes.data_as(pd), g.ctypes.data_as(pd),
                         e.ctypes.data_as(pd), 1e-3, 0, 0, None) == N.PF_ERR_ARG
    g[-1] = 0.0
    e[3] = -1.0
    assert L.pcr_prepare(C.byref(h), 8, a.ctypes.data_as(pd), g.ctypes.data_as(pd),
                         e.ctypes.data_as(pd), 1e-3, 0, 0, None) == N.PF_ERR_ARG
    e[3] = 0.0
    assert L.pcr_prepare(C.byref(h), 8, a.ctypes.data_as(pd), g.ctypes.data_as(pd),
                         e.ctypes.data_as(pd), -1.0, 0, 0, None) == N.PF_ERR_ARG
    assert L.pcr_prepare(C.byref(h), 8, a.ctypes.data_as(pd), g.ctypes.data_as(pd),
                         e.ctypes.data_as(pd), 1e-3, 0, 12, None) == N.PF_ERR_UNSUPPORTED
    big = 2000
    a2, g2, e2 = np.zeros(big), np.zeros(big), np.zeros(big)
    assert L.pcr_prepare(C.byref(h), big, a2.ctypes.data_as(pd), g2.ctypes.data_as(pd),
                         e2.ctypes.data_as(pd), 1e-3, 0, 32, None) == N.PF_ERR_UNSUPPORTED


def test_autotune_cache_ignores_corrupt_file(tmp_path):
    from paper_2502_06296_amd import autotune
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert autotune.load_cache(str(p)) == {}
    autotune.save_cache({"k": {"zsolve_variant": 3}}, str(p))
    assert autotune.load_cache(str(p)) == {"k": {"zsolve_variant": 3}}


def test_pcr_prepare_rows_rejects_rows_outside_the_m_matrix_form():
    """The (lower, diag, upper) form of L_z is validated and converted on the
    host before anything reaches the device."""
    L = N.lib()
    pd = C.POINTER(C.c_double)
    n = 8
    lo = np.full(n, 2.0); up = np.full(n, 3.0)
    lo[0] = 0.0; up[-1] = 0.0
    di = -(lo + up)
    h = C.c_void_p()

    def call(lo, di, up, s=1e-3):
        return L.pcr_prepare_rows(C.byref(h), n, lo.ctypes.data_as(pd), di.ctypes.data_as(pd),
                                  up.ctypes.data_as(pd), s, 0, 0, None)
    bad = lo.copy(); bad[0] = 1.0                     # coupling below the first row
    assert call(bad, di, up) == N.PF_ERR_ARG
    bad = up.copy(); bad[3] = -1.0                    # negative off-diagonal
    assert call(lo, di, bad) == N.PF_ERR_UNSUPPORTED
    bad = di.copy(); bad[4] = -4.0                    # |diag| below lower + upper = 5
    assert call(lo, bad, up) == N.PF_ERR_UNSUPPORTED
    bad = di.copy(); bad[2] = np.nan
    assert call(lo, bad, up) == N.PF_ERR_ARG
    assert call(lo, di, up, s=-1.0) == N.PF_ERR_ARG
    assert L.pcr_prepare_rows(C.byref(h), 3, lo.ctypes.data_as(pd), di.ctypes.data_as(pd),
                              up.ctypes.data_as(pd), 1e-3, 0, 0, None) == N.PF_ERR_ARG
    assert b"M-matrix" in L.pf_last_error() or L.pf_last_error()


def test_plan_validates_the_x_boundary_before_any_device_call():
    L = N.lib()
    h = C.c_void_p()
    g, keep = N.make_grid(64, 64, 64, 2 * np.pi, np.pi, 2.0, 1.5, None, 0, 4)
    assert L.poisson_plan(C.byref(h), C.byref(g), 0, 1, None, None) == N.PF_ERR_ARG
    g, keep = N.make_grid(64, 64, 64, 2 * np.pi, np.pi, 2.0, 1.5, None, 0, -1)
    assert L.poisson_plan(C.byref(h), C.byref(g), 0, 1, None, None) == N.PF_ERR_ARG
    assert L.pf_abi_version() == 3


def test_batched_calls_check_their_counts_before_any_device_call():
    L = N.lib()
    arr = (C.c_void_p * 17)()
    i32 = (C.c_int32 * 17)()
    assert L.pcr_apply_batched(0, arr, arr, i32, i32) == N.PF_ERR_ARG
    assert L.pcr_apply_batched(17, arr, arr, i32, i32) == N.PF_ERR_ARG      # 1..16 fields
    assert L.poisson_solve_batched(-1, arr, arr, arr) == N.PF_ERR_ARG
    assert L.poisson_solve_batched(0, arr, arr, arr) == N.PF_OK            # nothing to do
    assert L.poisson_solve_batched(1, arr, arr, arr) == N.PF_ERR_ARG       # NULL plan

