"""Python face of the C ABI, with the same names (include/pf_channel.h).

Fields are torch tensors on a HIP device, C-order (nz, ny, nx). Plans hold a
handle to the library's plan; workspaces are torch allocations the plan keeps
alive. Nothing here computes: every call goes to libpf_channel.so.
"""
from __future__ import annotations

import ctypes as C

from . import _native as N

PRECISIONS = {"fp64": N.PF_FP64, "fp32": N.PF_FP32, "fp32_refine": N.PF_FP32_REFINE}
BCS = {"neumann": N.PF_BC_NEUMANN, "dirichlet_centre": N.PF_BC_DIRICHLET_CENTRE,
       "dirichlet_face": N.PF_BC_DIRICHLET_FACE}


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def grid_faces(nx, ny, nz, lx=6.283185307179586, ly=3.141592653589793, lz=2.0, beta=1.5, zf=None):
    """Face coordinates the library uses for this grid (numpy, nz+1)."""
    import numpy as np
    g, keep = N.make_grid(nx, ny, nz, lx, ly, lz, beta, zf)
    out = np.empty(nz + 1, dtype=np.float64)
    N.check(N.lib().pf_grid_faces(C.byref(g), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def zop_rows(nz, bc, lz=2.0, beta=1.5, zf=None):
    """(alpha, gamma, excess) of -L_z for a boundary family (numpy arrays)."""
    import numpy as np
    bc = BCS[bc] if isinstance(bc, str) else int(bc)
    n = nz - 1 if bc == N.PF_BC_DIRICHLET_FACE else nz
    g, keep = N.make_grid(64, 64, nz, 1.0, 1.0, lz, beta, zf)
    a, b, c = (np.empty(n, dtype=np.float64) for _ in range(3))
    pd = C.POINTER(C.c_double)
    N.check(N.lib().pf_zop_rows(C.byref(g), bc, a.ctypes.data_as(pd), b.ctypes.data_as(pd),
                                c.ctypes.data_as(pd)))
    return a, b, c


class PoissonPlan:
    def __init__(self, handle, shape, precision, stream, workspace):
        self.handle = handle
        self.shape = shape
        self.precision = precision
        self.stream = stream
        self.workspace = workspace

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and N._lib is not None:
            N._lib.poisson_destroy(h)
            self.handle = None


YBCS = {"periodic": 0, "walls": 1, "dirichlet": 2, "faces": 3}


def poisson_plan(nx, ny, nz, lx=6.283185307179586, ly=3.141592653589793, lz=2.0, beta=1.5,
                 zf=None, precision="fp64", n_refine=1, stream=None, device=None, ybc="periodic",
                 xbc="periodic", tuned=True):
    """Plan the channel Poisson solve; allocates the workspace as a torch tensor.
    ybc "walls": zero-gradient walls at both y ends (cosine transform in y);
    "dirichlet": value-zero walls at both y ends (sine transform in y); xbc
    the same at both x ends. tuned: apply the autotuner's cached launch
    shapes for this grid and precision, if the cache holds them."""
    import torch
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    yb = YBCS[ybc] if isinstance(ybc, str) else int(ybc)
    xb = YBCS[xbc] if isinstance(xbc, str) else int(xbc)
    with torch.cuda.device(dev):
        g, keep = N.make_grid(nx, ny, nz, lx, ly, lz, beta, zf, yb, xb)
        h = C.c_void_p()
        ws = C.c_size_t(0)
        s = N.stream_handle(stream)
        N.check(N.lib().poisson_plan(C.byref(h), C.byref(g), _prec(precision), int(n_refine), s,
                                     C.byref(ws)))
        plan = PoissonPlan(h, (nz, ny, nx), _prec(precision), stream, None)
        if ws.value:
            plan.workspace = torch.empty(ws.value, dtype=torch.uint8, device=dev)
            N.check(N.lib().poisson_set_workspace(h, _ptr(plan.workspace), ws.value))
        if tuned:
            from . import autotune
            autotune.apply_cached_poisson(plan, nx, ny, nz, precision)
    return plan


def helmholtz3d_plan(nx, ny, nz, bc, s, lx=6.283185307179586, ly=3.141592653589793, lz=2.0, beta=1.5,
                     zf=None, precision="fp64", n_refine=1, stream=None, device=None, ybc="periodic",
                     xbc="periodic"):
    """Plan the 3-D implicit Helmholtz (I - s L) u = r (bc "dirichlet_centre":
    fields of nz planes; "dirichlet_face": nz - 1; ybc and xbc as for
    poisson_plan, for a field at cell-centre x and y positions; ybc "faces":
    a field on the y faces between value-zero walls, row ny - 1 the top wall
    face, zero in the result up to rounding); allocates the workspace."""
    import torch
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    b = BCS[bc] if isinstance(bc, str) else int(bc)
    yb = YBCS[ybc] if isinstance(ybc, str) else int(ybc)
    xb = YBCS[xbc] if isinstance(xbc, str) else int(xbc)
    with torch.cuda.device(dev):
        g, keep = N.make_grid(nx, ny, nz, lx, ly, lz, beta, zf, yb, xb)
        h = C.c_void_p()
        ws = C.c_size_t(0)
        N.check(N.lib().helmholtz3d_plan(C.byref(h), C.byref(g), b, float(s), _prec(precision),
                                         int(n_refine), N.stream_handle(stream), C.byref(ws)))
        n = nz - 1 if b == N.PF_BC_DIRICHLET_FACE else nz
        plan = PoissonPlan(h, (n, ny, nx), _prec(precision), stream, None)
        if ws.value:
            plan.workspace = torch.empty(ws.value, dtype=torch.uint8, device=dev)
            N.check(N.lib().poisson_set_workspace(h, _ptr(plan.workspace), ws.value))
    return plan


def helmholtz3d_solve(plan, r, u):
    """u <- (I - s L)^{-1} r (float64 device tensors of the plan's shape)."""
    import torch
    _check_field(r, plan.shape, torch.float64)
    _check_field(u, plan.shape, torch.float64)
    N.check(N.lib().helmholtz3d_solve(plan.handle, _ptr(r), _ptr(u)))
    return u


def helmholtz3d_update(plan, s):
    N.check(N.lib().helmholtz3d_update(plan.handle, float(s)))


def _check_field(t, shape, dtype):
    import torch
    if not t.is_cuda or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor of shape {shape}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    return torch


def poisson_solve(plan, rhs, p):
    """p <- L7^{-1} rhs (float64 device tensors of the plan's shape)."""
    import torch
    _check_field(rhs, plan.shape, torch.float64)
    _check_field(p, plan.shape, torch.float64)
    N.check(N.lib().poisson_solve(plan.handle, _ptr(rhs), _ptr(p)))
    return p


def poisson_solve_noalloc(plan, rhs, p):
    """poisson_solve with the library's static device scratch as the work
    arrays (no allocation; calls on one GPU must not overlap in time)."""
    import torch
    _check_field(rhs, plan.shape, torch.float64)
    _check_field(p, plan.shape, torch.float64)
    N.check(N.lib().poisson_solve_noalloc(plan.handle, _ptr(rhs), _ptr(p)))
    return p


def poisson_set_status(plan, status, tol=1e-10):
    """Record the a-posteriori status of the plan's solves into `status`, a
    device int64 tensor of 4 elements (None stops recording)."""
    import torch
    if status is not None:
        if not status.is_cuda or status.dtype != torch.int64 or status.numel() != 4 or not status.is_contiguous():
            raise ValueError("status must be a contiguous cuda int64 tensor of 4 elements")
    N.check(N.lib().poisson_set_status(plan.handle, _ptr(status) if status is not None else None, float(tol)))
    plan.status = status


def read_status(status):
    """(est_rel_err, flags) of a status tensor (synchronises with its stream)."""
    v = status.cpu()
    return float(v[2:3].view(__import__("torch").float64)[0]), int(v[3])


def poisson_project(plan, u, v, w, p, phi, gdt, c=0.0):
    """Pressure projection: L7 phi = D u* / gdt, u <- u* - gdt G phi, p <- p +
    phi - c L_z phi. u, v, p, phi: float64 (nz, ny, nx); w: float64 (nz-1,
    ny, nx) on the interior z faces. u, v, w, p are updated in place; phi
    receives the correction pressure."""
    import torch
    nz, ny, nx = plan.shape
    for t in (u, v, p, phi):
        _check_field(t, plan.shape, torch.float64)
    _check_field(w, (nz - 1, ny, nx), torch.float64)
    N.check(N.lib().poisson_project(plan.handle, _ptr(u), _ptr(v), _ptr(w), _ptr(p), _ptr(phi),
                                    float(gdt), float(c)))
    return phi


def poisson_solve_batched(plans, rhs, p):
    import torch
    n = len(plans)
    for pl, r, q in zip(plans, rhs, p):
        _check_field(r, pl.shape, torch.float64)
        _check_field(q, pl.shape, torch.float64)
    arr = C.c_void_p * n
    N.check(N.lib().poisson_solve_batched(n, arr(*[pl.handle for pl in plans]),
                                          arr(*[r.data_ptr() for r in rhs]),
                                          arr(*[q.data_ptr() for q in p])))


def poisson_set_stream(plan, stream):
    N.check(N.lib().poisson_set_stream(plan.handle, N.stream_handle(stream)))
    plan.stream = stream


class PcrPlan:
    def __init__(self, handle, n, precision, stream):
        self.handle = handle
        self.n = n
        self.precision = precision
        self.stream = stream

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and N._lib is not None:
            N._lib.pcr_destroy(h)
            self.handle = None


def pcr_prepare(alpha, gamma, excess, s, precision="fp64", chunk_rows=0, stream=None):
    """Algorithm 2, Step 1 for (I - s L_z); alpha, gamma, excess: host rows of -L_z."""
    import numpy as np
    a, b, c = (np.ascontiguousarray(v, dtype=np.float64) for v in (alpha, gamma, excess))
    n = a.size
    pd = C.POINTER(C.c_double)
    h = C.c_void_p()
    N.check(N.lib().pcr_prepare(C.byref(h), n, a.ctypes.data_as(pd), b.ctypes.data_as(pd),
                                c.ctypes.data_as(pd), float(s), _prec(precision), int(chunk_rows),
                                N.stream_handle(stream)))
    return PcrPlan(h, n, _prec(precision), stream)


def pcr_prepare_rows(lower, diag, upper, s, precision="fp64", chunk_rows=0, stream=None):
    """The same plan from the rows (lower, diag, upper) of L_z itself."""
    import numpy as np
    a, b, c = (np.ascontiguousarray(v, dtype=np.float64) for v in (lower, diag, upper))
    n = a.size
    pd = C.POINTER(C.c_double)
    h = C.c_void_p()
    N.check(N.lib().pcr_prepare_rows(C.byref(h), n, a.ctypes.data_as(pd), b.ctypes.data_as(pd),
                                     c.ctypes.data_as(pd), float(s), _prec(precision), int(chunk_rows),
                                     N.stream_handle(stream)))
    return PcrPlan(h, n, _prec(precision), stream)


def pcr_update_coef(plan, s):
    N.check(N.lib().pcr_update_coef(plan.handle, float(s)))


def _pcr_dtype(plan):
    import torch
    return torch.float32 if plan.precision == N.PF_FP32 else torch.float64


def pcr_apply(plan, field):
    """In-place Helmholtz solve of every column of field (n, ny, nx)."""
    n, ny, nx = field.shape
    if n != plan.n:
        raise ValueError(f"field has {n} rows, plan has {plan.n}")
    _check_field(field, field.shape, _pcr_dtype(plan))
    N.check(N.lib().pcr_apply(plan.handle, _ptr(field), nx, ny))
    return field


def pcr_apply_batched(plans, fields):
    n = len(plans)
    for pl, f in zip(plans, fields):
        if f.shape[0] != pl.n:
            raise ValueError("field rows do not match plan")
        _check_field(f, f.shape, _pcr_dtype(pl))
    vp = C.c_void_p * n
    i32 = C.c_int32 * n
    N.check(N.lib().pcr_apply_batched(n, vp(*[p.handle for p in plans]),
                                      vp(*[f.data_ptr() for f in fields]),
                                      i32(*[f.shape[2] for f in fields]),
                                      i32(*[f.shape[1] for f in fields])))


def pcr_set_stream(plan, stream):
    N.check(N.lib().pcr_set_stream(plan.handle, N.stream_handle(stream)))
    plan.stream = stream


# -------------------------------------------------------------- task batch
def _task_array(tasks):
    """The pf_task array of a list of task dicts (see run_batched)."""
    import torch
    arr = (N.PfTask * max(1, len(tasks)))()
    for t, task in enumerate(tasks):
        T = arr[t]
        pl = task.get("poisson")
        if pl is not None:
            _check_field(task["rhs"], pl.shape, torch.float64)
            _check_field(task["p"], pl.shape, torch.float64)
            T.poisson, T.rhs, T.p = pl.handle, task["rhs"].data_ptr(), task["p"].data_ptr()
        plans, fields = task.get("pcr", []), task.get("fields", [])
        if len(plans) != len(fields) or len(plans) > 4:
            raise ValueError("a task takes up to 4 Helmholtz plans with one field each")
        T.ncomp = len(plans)
        for c, (hp, f) in enumerate(zip(plans, fields)):
            if f.shape[0] != hp.n:
                raise ValueError("field rows do not match plan")
            _check_field(f, f.shape, _pcr_dtype(hp))
            T.pcr[c], T.field[c] = hp.handle, f.data_ptr()
            T.nx[c], T.ny[c] = f.shape[2], f.shape[1]
    return arr


def run_batched(tasks, lanes=4, stream=None):
    """Independent tasks spread over `lanes` internal streams forked from and
    joined back into `stream` (pf_run_batched). Each task is a dict with an
    optional Poisson solve (``poisson``, ``rhs``, ``p``) and an optional group
    of up to 4 Helmholtz fields (``pcr``: plans, ``fields``: tensors)."""
    arr = _task_array(tasks)
    N.check(N.lib().pf_run_batched(len(tasks), arr, int(lanes), N.stream_handle(stream)))


# ------------------------------------------------------------------ graphs
class Graph:
    def __init__(self, handle):
        self.handle = handle

    def launch(self, stream):
        N.check(N.lib().pf_graph_launch(self.handle, N.stream_handle(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and N._lib is not None:
            N._lib.pf_graph_destroy(h)
            self.handle = None


def pf_graph_begin(stream):
    N.check(N.lib().pf_graph_begin(N.stream_handle(stream)))


def pf_graph_end(stream):
    h = C.c_void_p()
    N.check(N.lib().pf_graph_end(N.stream_handle(stream), C.byref(h)))
    return Graph(h)


# ------------------------------------------------------------- measurement
def poisson_timing(plan, enable=True):
    N.check(N.lib().poisson_timing(plan.handle, 1 if enable else 0))


def _read(fn, handle):
    ms = (C.c_double * N.PF_STAGE_COUNT)()
    cnt = (C.c_int32 * N.PF_STAGE_COUNT)()
    N.check(fn(handle, ms, cnt))
    return {N.STAGES[i]: (ms[i], cnt[i]) for i in range(N.PF_STAGE_COUNT) if cnt[i]}


def poisson_timing_read(plan):
    """{stage: (summed ms, launches)} since the last read (synchronises)."""
    return _read(N.lib().poisson_timing_read, plan.handle)


def pcr_timing(plan, enable=True):
    N.check(N.lib().pcr_timing(plan.handle, 1 if enable else 0))


def pcr_timing_read(plan):
    return _read(N.lib().pcr_timing_read, plan.handle)


def pf_copy_kernel(dst, src, stream=None):
    nbytes = src.numel() * src.element_size()
    N.check(N.lib().pf_copy_kernel(_ptr(dst), _ptr(src), nbytes, N.stream_handle(stream)))
