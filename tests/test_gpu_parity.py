"""HIP path against the CPU oracle, element by element, through the C ABI.

Bars: float64 1e-12; float32 with one float64-residual correction 1e-10;
plain float32 1e-5 (reported, no accuracy claim). Each bar holds for the
relative L2 error over all points and for the largest element-wise error
against the largest reference value. Shapes span several tiles and ragged
tails: z lengths that are not multiples of the 16-row chunk, radix-3 and
radix-5 lengths, the largest x and y lengths, the x, y and z lengths of the
1024x512x512 and 2048x1024x1024 workloads (the same kernel instances and
z-solve shapes as there), both z-solve layouts (more than 32 chunks per
column switches to 8-column workgroups) and both Helmholtz layouts (more
than 16 chunks switches to 32-column chunks).
"""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
import synth
from oracle import grid as ogrid
from oracle import poisson as op
from parity import check

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi
S_C3 = 0.5 * (1.0 / 5200.0) * 1e-4
TOL = {"fp64": 1e-12, "fp32_refine": 1e-10, "fp32": 1e-5}


def _dev():
    return torch.device("cuda", 0)


def _solve_gpu(f, zf, prec, beta=None, use_zf=True):
    nz, ny, nx = f.shape
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta if beta is not None else 1.5,
                           zf=zf if use_zf else None, precision=prec)
    rhs = torch.from_numpy(f).to(_dev())
    p = torch.empty_like(rhs)
    pf.poisson_solve(plan, rhs, p)
    torch.cuda.synchronize()
    return p.cpu().numpy()


POISSON_SHAPES = [
    (64, 64, 64, 1.5, 0),       # the 64^3 channel case
    (128, 96, 40, 2.0, 1),      # radix-3 y, ragged z chunks
    (192, 256, 33, 1.0, 2),     # radix-3 x, nz = 2*16 + 1
    (256, 192, 128, 0.0, 3),    # uniform z
    (96, 64, 520, 1.5, 4),      # more than 32 z chunks: 8-column workgroups
    (2048, 64, 8, 1.5, 5),      # largest x length, single chunk
    (64, 2048, 6, 1.2, 6),      # largest y length
    (384, 768, 20, 1.5, 7),
    (1536, 128, 17, 1.8, 8),
    (128, 1024, 4, 1.5, 9),     # smallest nz
    (64, 64, 1024, 1.5, 10),    # largest nz: the z solve falls back to a shape that fits the LDS
    (3456, 64, 30, 1.5, 11),    # the weak-scaling share's lengths: x = 3456 (2^7 3^3)
    (3072, 64, 30, 1.5, 12),    # x = 3072
    (64, 3072, 30, 1.5, 13),    # y = 3072
    (3200, 64, 28, 1.5, 14),    # the strong-scaling grid's x length 3200 = 2^7 5^2: radix-5 passes
    (64, 3456, 28, 1.5, 15),    # its y length 3456, six-wave y workgroups
    (128, 3200, 9, 1.5, 16),    # radix 5 along y, five-wave y workgroups
    (1024, 512, 24, 1.5, 17),   # the 1024x512x512 workload's x and y lengths
    (2048, 1024, 8, 1.5, 18),   # the 2048x1024x1024 workload's x and y lengths
    # the z lengths of the two workloads: the z-solve shape depends on nx only
    # through divisibility by its columns per workgroup (at most 128), so
    # these run the workloads' own z-solve kernels
    (256, 64, 512, 1.5, 19),
    (128, 64, 1024, 1.5, 20),
]


@pytest.mark.parametrize("nx,ny,nz,beta,seed", POISSON_SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_poisson_matches_oracle(nx, ny, nz, beta, seed, prec):
    print(f"poisson {prec} {nx}x{ny}x{nz} beta={beta} seed={seed}", flush=True)
    f, zf = synth.channel_rhs(seed, nx, ny, nz, beta=beta)
    ref = op.solve_poisson(f, zf, LX, LY)
    got = _solve_gpu(f, zf, prec)
    check(got, ref, TOL[prec], prec)


def test_poisson_tanh_faces_built_in_library():
    """zf = NULL: the library's own tanh faces give the oracle's solution."""
    f, zf = synth.channel_rhs(12, 128, 64, 48, beta=1.5)
    ref = op.solve_poisson(f, zf, LX, LY)
    got = _solve_gpu(f, zf, "fp64", beta=1.5, use_zf=False)
    check(got, ref, 1e-12, "fp64")


def test_poisson_incompatible_rhs_is_projected():
    f, zf = synth.channel_rhs(13, 64, 64, 32, beta=1.5)
    f = f + 0.25
    ref = op.solve_poisson(f, zf, LX, LY)
    for prec in ("fp64", "fp32_refine"):
        got = _solve_gpu(f, zf, prec)
        check(got, ref, TOL[prec], prec)
        w = np.diff(zf)
        assert abs(np.sum(got * w[:, None, None])) < 1e-10 * np.sum(np.abs(got) * w[:, None, None])


def test_poisson_zero_rhs_gives_zero():
    nx, ny, nz = 64, 64, 16
    zf = synth.tanh_faces(nz)
    for prec in ("fp64", "fp32_refine"):
        got = _solve_gpu(np.zeros((nz, ny, nx)), zf, prec)
        assert np.all(got == 0.0)


def test_poisson_mid_size_like_full_case():
    """Same z length and stretching as the 1024x512x512 case, smaller plane."""
    nx, ny, nz = 256, 128, 512
    f, zf = synth.channel_rhs(21, nx, ny, nz, beta=1.5)
    ref = op.solve_poisson(f, zf, LX, LY)
    for prec in ("fp64", "fp32_refine"):
        got = _solve_gpu(f, zf, prec)
        check(got, ref, TOL[prec], f"poisson {prec} {nx}x{ny}x{nz}")


def test_poisson_deterministic():
    f, zf = synth.channel_rhs(5, 128, 128, 64, beta=1.5)
    for prec in ("fp64", "fp32_refine"):
        a = _solve_gpu(f, zf, prec)
        b = _solve_gpu(f, zf, prec)
        np.testing.assert_array_equal(a, b)


# --------------------------------------------------------------- Helmholtz
HELM_CASES = [
    (64, 64, 64, ogrid.DIRICHLET_CENTRE),
    (64, 64, 64, ogrid.DIRICHLET_FACE),
    (128, 32, 40, ogrid.DIRICHLET_CENTRE),     # ragged chunk
    (192, 8, 33, ogrid.DIRICHLET_FACE),        # 32 unknowns
    (64, 16, 512, ogrid.DIRICHLET_CENTRE),     # 16 chunks of 32 rows
    (64, 16, 512, ogrid.DIRICHLET_FACE),       # 511 unknowns
    (128, 4, 1000, ogrid.DIRICHLET_CENTRE),    # more than 16 chunks: 32-column layout
    (64, 2, 5, ogrid.DIRICHLET_CENTRE),        # 5 unknowns, one chunk
    (3456, 2, 30, ogrid.DIRICHLET_FACE),       # the weak-scaling share's x length and nz
    (64, 4, 1024, ogrid.DIRICHLET_CENTRE),     # the 2048x1024x1024 workload's columns: 32 chunks
    (64, 4, 1024, ogrid.DIRICHLET_FACE),       # its w columns, 1023 unknowns
]


def _helm(r, zf, s, bc, prec, chunk_rows=0):
    al, ga, ex = ogrid.zop(zf, bc)
    plan = pf.pcr_prepare(al, ga, ex, s, precision=prec, chunk_rows=chunk_rows)
    dt = torch.float32 if prec == "fp32" else torch.float64
    u = torch.from_numpy(r).to(_dev(), dt)
    pf.pcr_apply(plan, u)
    torch.cuda.synchronize()
    return u.double().cpu().numpy()


@pytest.mark.parametrize("nx,ny,nz,bc", HELM_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
@pytest.mark.parametrize("s", [S_C3, 1e-2])
def test_helmholtz_matches_oracle(nx, ny, nz, bc, prec, s):
    print(f"helmholtz {prec} {nx}x{ny}x{nz} bc={bc} s={s}", flush=True)
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    n = nz if bc == ogrid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(3, (n, ny, nx))
    ref = op.solve_helmholtz(r, zf, s, bc)
    got = _helm(r, zf, s, bc, prec)
    check(got, ref, TOL[prec], prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("nz,chunk_rows", [(200, 8), (200, 16), (200, 32), (64, 8), (128, 8), (512, 32)])
def test_helmholtz_chunkings_agree(nz, chunk_rows, prec):
    # s = 1e-2 couples the chunks strongly: the refinement's residual must see
    # exactly the chunk-end values that the neighbouring chunks store
    print(f"helmholtz {prec} nz={nz} chunk_rows={chunk_rows}", flush=True)
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    r = synth.normal01(4, (nz, 4, 64))
    ref = op.solve_helmholtz(r, zf, 1e-2, ogrid.DIRICHLET_CENTRE)
    got = _helm(r, zf, 1e-2, ogrid.DIRICHLET_CENTRE, prec, chunk_rows)
    check(got, ref, TOL[prec], prec)


def test_helmholtz_s_zero_is_identity():
    zf = synth.tanh_faces(48)
    r = synth.normal01(6, (48, 4, 64))
    got = _helm(r, zf, 0.0, ogrid.DIRICHLET_CENTRE, "fp64")
    np.testing.assert_array_equal(got, r)


def test_helmholtz_batched_three_components_equal_single():
    nx, ny, nz = 128, 8, 96
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    specs = [(ogrid.DIRICHLET_CENTRE, nz), (ogrid.DIRICHLET_CENTRE, nz), (ogrid.DIRICHLET_FACE, nz - 1)]
    for prec in ("fp64", "fp32_refine", "fp32"):
        dt = torch.float32 if prec == "fp32" else torch.float64
        plans, fields, singles = [], [], []
        for c, (bc, n) in enumerate(specs):
            al, ga, ex = ogrid.zop(zf, bc)
            plans.append(pf.pcr_prepare(al, ga, ex, S_C3, precision=prec))
            r = synth.normal01(10 + c, (n, ny, nx))
            fields.append(torch.from_numpy(r).to(_dev(), dt))
            singles.append(torch.from_numpy(r).to(_dev(), dt))
        pf.pcr_apply_batched(plans, fields)
        for pl, s1 in zip(plans, singles):
            pf.pcr_apply(pl, s1)
        torch.cuda.synchronize()
        for a, b in zip(fields, singles):
            assert torch.equal(a, b)


def test_pcr_update_coef_matches_fresh_plan():
    nz = 64
    zf = synth.tanh_faces(nz)
    al, ga, ex = ogrid.zop(zf, ogrid.DIRICHLET_CENTRE)
    r = synth.normal01(8, (nz, 4, 64))
    plan = pf.pcr_prepare(al, ga, ex, 1e-3, precision="fp64")
    pf.pcr_update_coef(plan, 2e-2)
    u = torch.from_numpy(r).to(_dev())
    pf.pcr_apply(plan, u)
    torch.cuda.synchronize()
    ref = op.solve_helmholtz(r, zf, 2e-2, ogrid.DIRICHLET_CENTRE)
    check(u.cpu().numpy(), ref, 1e-12, "fp64")


# ------------------------------------------------------------------ errors
def test_solve_rejects_overlap_and_missing_workspace():
    import ctypes as C
    from paper_2502_06296_amd import _native as N
    plan = pf.poisson_plan(64, 64, 16, precision="fp64")
    a = torch.zeros((16, 64, 64), dtype=torch.float64, device=_dev())
    with pytest.raises(N.PfError) as e:
        N.check(N.lib().poisson_solve(plan.handle, C.c_void_p(a.data_ptr()), C.c_void_p(a.data_ptr())))
    assert e.value.code == N.PF_ERR_ARG
    plan2 = pf.poisson_plan(64, 64, 16, precision="fp32_refine")
    N.check(N.lib().poisson_set_workspace(plan2.handle, None, 0)) if False else None
    b = torch.zeros_like(a)
    with pytest.raises(N.PfError):
        N.check(N.lib().poisson_set_workspace(plan2.handle, C.c_void_p(b.data_ptr()), 16))
