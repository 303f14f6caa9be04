"""ctypes binding of libpf_channel.so (declared in include/pf_channel.h).

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch provides device memory (tensors) and streams; a missing library is
an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libpf_channel.so")

PF_OK, PF_ERR_ARG, PF_ERR_UNSUPPORTED, PF_ERR_DEVICE, PF_ERR_WORKSPACE = 0, -1, -2, -3, -4
PF_FP64, PF_FP32, PF_FP32_REFINE = 0, 1, 2
PF_BC_NEUMANN, PF_BC_DIRICHLET_CENTRE, PF_BC_DIRICHLET_FACE = 0, 1, 2
STAGES = ["xfwd", "yfwd", "zsolve", "yinv", "xinv", "zero_mode", "xfwd_resid", "xinv_final",
          "pcr_apply", "project"]
PF_STAGE_COUNT = len(STAGES)

# every symbol include/pf_channel.h declares
EXPORTS = [
    "pf_last_error", "pf_abi_version", "pf_zop_rows", "pf_grid_faces",
    "poisson_plan", "poisson_set_workspace", "poisson_solve", "poisson_solve_noalloc", "poisson_project",
    "poisson_solve_batched",
    "helmholtz3d_plan", "helmholtz3d_solve", "helmholtz3d_update", "poisson_set_status",
    "poisson_set_stream", "poisson_destroy",
    "pcr_prepare", "pcr_prepare_rows", "pcr_update_coef", "pcr_apply", "pcr_apply_batched", "pcr_set_stream",
    "pcr_destroy",
    "pf_graph_begin", "pf_graph_end", "pf_graph_launch", "pf_graph_destroy",
    "poisson_timing", "poisson_timing_read", "pcr_timing", "pcr_timing_read",
    "pf_copy_kernel",
    "poisson_variant_count", "poisson_set_variant", "poisson_get_variant",
    "pcr_set_shape", "pcr_get_shape",
    "pf_run_batched",
]


class PfGrid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("beta", C.c_double), ("zf", C.POINTER(C.c_double)), ("ybc", C.c_int32),
                ("xbc", C.c_int32)]


class PfTask(C.Structure):
    _fields_ = [("poisson", C.c_void_p), ("rhs", C.c_void_p), ("p", C.c_void_p),
                ("ncomp", C.c_int32), ("pcr", C.c_void_p * 4), ("field", C.c_void_p * 4),
                ("nx", C.c_int32 * 4), ("ny", C.c_int32 * 4)]


class PfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pf status {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library missing: {LIB_PATH}. Build it with "
                "`python -m paper_2502_06296_amd.build` (hipcc, gfx950).")
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl, sz = C.c_void_p, C.c_int32, C.c_double, C.c_size_t
        pd = C.POINTER(C.c_double)
        sig = {
            "pf_last_error": (C.c_char_p, []),
            "pf_abi_version": (i32, []),
            "pf_zop_rows": (i32, [C.POINTER(PfGrid), i32, pd, pd, pd]),
            "pf_grid_faces": (i32, [C.POINTER(PfGrid), pd]),
            "poisson_plan": (i32, [C.POINTER(vp), C.POINTER(PfGrid), i32, i32, vp, C.POINTER(sz)]),
            "poisson_set_workspace": (i32, [vp, vp, sz]),
            "poisson_solve": (i32, [vp, vp, vp]),
            "poisson_solve_noalloc": (i32, [vp, vp, vp]),
            "poisson_project": (i32, [vp, vp, vp, vp, vp, vp, C.c_double, C.c_double]),
            "helmholtz3d_plan": (i32, [C.POINTER(vp), C.POINTER(PfGrid), i32, C.c_double, i32, i32, vp,
                                       C.POINTER(sz)]),
            "helmholtz3d_solve": (i32, [vp, vp, vp]),
            "poisson_set_status": (i32, [vp, vp, C.c_double]),
            "helmholtz3d_update": (i32, [vp, C.c_double]),
            "poisson_solve_batched": (i32, [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)]),
            "poisson_set_stream": (i32, [vp, vp]),
            "poisson_destroy": (i32, [vp]),
            "pcr_prepare": (i32, [C.POINTER(vp), i32, pd, pd, pd, dbl, i32, i32, vp]),
            "pcr_prepare_rows": (i32, [C.POINTER(vp), i32, pd, pd, pd, dbl, i32, i32, vp]),
            "pcr_update_coef": (i32, [vp, dbl]),
            "pcr_apply": (i32, [vp, vp, i32, i32]),
            "pcr_apply_batched": (i32, [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(i32),
                                        C.POINTER(i32)]),
            "pcr_set_stream": (i32, [vp, vp]),
            "pcr_destroy": (i32, [vp]),
            "pf_graph_begin": (i32, [vp]),
            "pf_graph_end": (i32, [vp, C.POINTER(vp)]),
            "pf_graph_launch": (i32, [vp, vp]),
            "pf_graph_destroy": (i32, [vp]),
            "poisson_timing": (i32, [vp, i32]),
            "poisson_timing_read": (i32, [vp, pd, C.POINTER(i32)]),
            "pcr_timing": (i32, [vp, i32]),
            "pcr_timing_read": (i32, [vp, pd, C.POINTER(i32)]),
            "pf_copy_kernel": (i32, [vp, vp, sz, vp]),
            "poisson_variant_count": (i32, [vp, i32, C.POINTER(i32)]),
            "poisson_set_variant": (i32, [vp, i32, i32]),
            "poisson_get_variant": (i32, [vp, i32, C.POINTER(i32)]),
            "pcr_set_shape": (i32, [vp, i32, i32]),
            "pcr_get_shape": (i32, [vp, C.POINTER(i32), C.POINTER(i32)]),
            "pf_run_batched": (i32, [i32, C.POINTER(PfTask), i32, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != PF_OK:
        raise PfError(code, lib().pf_last_error().decode())


def make_grid(nx, ny, nz, lx=6.283185307179586, ly=3.141592653589793, lz=2.0, beta=1.5, zf=None,
              ybc=0, xbc=0):
    """(PfGrid, keep-alive) for the C ABI; zf is an optional host array of nz+1 faces;
    ybc and xbc: 0 periodic, 1 zero-gradient walls, 2 value-zero walls; ybc 3:
    a field on the y faces between value-zero walls."""
    keep = None
    zp = None
    if zf is not None:
        import numpy as np
        keep = np.ascontiguousarray(zf, dtype=np.float64)
        if keep.shape != (nz + 1,):
            raise ValueError("zf must have nz+1 entries")
        zp = keep.ctypes.data_as(C.POINTER(C.c_double))
    return PfGrid(nx, ny, nz, lx, ly, lz, beta, zp, ybc, xbc), keep


def stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)
