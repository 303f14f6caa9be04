"""Poisson solve with walls at both y ends -- zero-gradient (the cosine
transform of Sec. 2.2.1 along y) and value-zero (the sine transform) --
through the C ABI against the CPU oracle, element by element, in the three
precisions, for the Poisson solve, the 3-D Helmholtz and (zero-gradient
walls) the projection.

Bars: float64 1e-12, float32 with one float64-residual correction 1e-10,
plain float32 1e-5, each for the relative L2 error and for the largest
element-wise error against the largest reference value.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
from paper_2502_06296_amd import _native as N
import synth
from oracle import grid as ogrid
from oracle import poisson as op
from parity import check

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi
TOL = {"fp64": 1e-12, "fp32_refine": 1e-10, "fp32": 1e-5}


def _dev():
    return torch.device("cuda", 0)


YBC = {"walls": ogrid.Y_WALLS, "dirichlet": ogrid.Y_DIRICHLET}


def _solve_gpu(f, zf, beta, prec, ybc="walls"):
    nz, ny, nx = f.shape
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta, zf=zf, precision=prec, ybc=ybc)
    rhs = torch.from_numpy(f).to(_dev())
    p = torch.empty_like(rhs)
    pf.poisson_solve(plan, rhs, p)
    torch.cuda.synchronize()
    return p.cpu().numpy()


CASES = [
    (64, 64, 64, 1.5, 0),      # the 64^3 channel with y walls
    (128, 96, 40, 2.0, 1),     # radix-3 y, ragged z chunks
    (256, 192, 33, 0.0, 2),    # uniform z
    (96, 128, 9, 1.2, 3),
    (64, 2048, 6, 1.5, 4),     # long y lines
    (64, 3200, 5, 1.5, 5),     # radix-5 y
    (1024, 512, 8, 1.5, 6),    # the 1024x512x512 workload's x and y lengths
    (2048, 1024, 4, 1.5, 7),   # the 2048x1024x1024 workload's x and y lengths
]


@pytest.mark.parametrize("nx,ny,nz,beta,seed", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
@pytest.mark.parametrize("ybc", ["walls", "dirichlet"])
def test_ywalls_poisson_matches_oracle(nx, ny, nz, beta, seed, prec, ybc):
    print(f"y {ybc} {prec} {nx}x{ny}x{nz} beta={beta} seed={seed}", flush=True)
    zf = synth.tanh_faces(nz, 2.0, beta)
    f = synth.uniform_pm1(300 + seed, (nz, ny, nx))
    ref = op.solve_poisson(f, zf, LX, LY, ybc=YBC[ybc])
    got = _solve_gpu(f, zf, beta, prec, ybc)
    check(got, ref, TOL[prec], prec)


@pytest.mark.parametrize("ybc", ["walls", "dirichlet"])
def test_ywalls_residual_at_512x256x64(ybc):
    nx, ny, nz, beta = 512, 256, 64, 1.5
    zf = synth.tanh_faces(nz, 2.0, beta)
    f = synth.uniform_pm1(310, (nz, ny, nx))
    p64 = _solve_gpu(f, zf, beta, "fp64", ybc)
    r = op.residual7(p64, f, zf, LX, LY, ybc=YBC[ybc])
    res = np.max(np.abs(r)) / np.max(np.abs(f))
    print(f"fp64 7-point residual {res:.2e}", flush=True)
    assert res < 1e-12
    p32 = _solve_gpu(f, zf, beta, "fp32_refine", ybc)
    err = op.rel_l2(p32, p64)
    print(f"fp32_refine vs fp64 {err:.2e}", flush=True)
    assert err < 1e-10


def test_projection_rejects_value_zero_y_walls():
    nx, ny, nz = 64, 64, 16
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, ybc="dirichlet")
    t = [torch.zeros((nz if i != 2 else nz - 1, ny, nx), dtype=torch.float64, device=_dev())
         for i in range(5)]
    with pytest.raises(N.PfError) as e:
        pf.poisson_project(plan, t[0], t[1], t[2], t[3], t[4], 0.1, 0.0)
    assert e.value.code == N.PF_ERR_UNSUPPORTED


H3D_CASES = [
    (64, 64, 32, 1.5, ogrid.DIRICHLET_CENTRE, 1e-3, 0),
    (128, 96, 40, 2.0, ogrid.DIRICHLET_FACE, 0.05, 1),     # radix-3 y, ragged chunks
    (96, 3200, 6, 1.2, ogrid.DIRICHLET_CENTRE, 1e-2, 2),   # radix-5 y lines
    (1024, 512, 6, 1.5, ogrid.DIRICHLET_FACE, 1e-3, 3),    # the 1024x512x512 workload's lengths
]
H3D_BC = {ogrid.DIRICHLET_CENTRE: "dirichlet_centre", ogrid.DIRICHLET_FACE: "dirichlet_face"}


@pytest.mark.parametrize("nx,ny,nz,beta,bc,s,seed", H3D_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
@pytest.mark.parametrize("ybc", ["walls", "dirichlet"])
def test_ywalls_helmholtz3d_matches_oracle(nx, ny, nz, beta, bc, s, seed, prec, ybc):
    print(f"helmholtz3d y {ybc} {prec} {nx}x{ny}x{nz} bc={bc} s={s}", flush=True)
    zf = synth.tanh_faces(nz, 2.0, beta)
    n = nz if bc == ogrid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(320 + seed, (n, ny, nx))
    ref = op.solve_helmholtz3d(r, zf, s, bc, LX, LY, ybc=YBC[ybc])
    plan = pf.helmholtz3d_plan(nx, ny, nz, H3D_BC[bc], s, LX, LY, 2.0, beta, zf=zf, precision=prec,
                               ybc=ybc)
    rt = torch.from_numpy(r).to(_dev())
    u = torch.empty_like(rt)
    pf.helmholtz3d_solve(plan, rt, u)
    torch.cuda.synchronize()
    check(u.cpu().numpy(), ref, TOL[prec], prec)


@pytest.mark.parametrize("ybc", ["walls", "dirichlet"])
def test_ywalls_graph_replays_equal_eager(ybc):
    """The wall transforms keep the solve capturable: three replays of one
    captured FP32+refine solve, with eager work between them, equal the eager
    solve bitwise."""
    nx, ny, nz = 128, 96, 40
    stream = torch.cuda.Stream(device=_dev())
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine",
                           stream=stream, ybc=ybc)
    rhs = torch.from_numpy(synth.uniform_pm1(330, (nz, ny, nx))).to(_dev())
    pe = torch.empty_like(rhs)
    p = torch.empty_like(rhs)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        pf.poisson_solve(plan, rhs, pe)
    stream.synchronize()
    pf.pf_graph_begin(stream)
    pf.poisson_solve(plan, rhs, p)
    g = pf.pf_graph_end(stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            p.fill_(-1.0)
        g.launch(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(p, pe), rep


PROJ_CASES = [
    (64, 64, 64, 1.5, 0.0, 0),
    (128, 96, 40, 2.0, 1e-3, 1),   # radix-3 y, implicit z-diffusion pressure term
    (96, 128, 9, 1.2, 0.0, 2),
]


@pytest.mark.parametrize("nx,ny,nz,beta,c,seed", PROJ_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_ywalls_projection_matches_oracle(nx, ny, nz, beta, c, seed, prec):
    from oracle import projection as oproj
    print(f"projection y walls {prec} {nx}x{ny}x{nz} c={c}", flush=True)
    zf = synth.tanh_faces(nz, 2.0, beta)
    u = synth.uniform_pm1(340 + seed, (nz, ny, nx))
    v = synth.uniform_pm1(341 + seed, (nz, ny, nx))
    w = synth.uniform_pm1(342 + seed, (nz - 1, ny, nx))
    p = synth.uniform_pm1(343 + seed, (nz, ny, nx))
    gdt = 0.37
    ref = oproj.project(u, v, w, p, zf, LX, LY, gdt, c, ybc=ogrid.Y_WALLS)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta, zf=zf, precision=prec, ybc="walls")
    t = [torch.from_numpy(a).to(_dev()) for a in (u, v, w, p)]
    phi = torch.empty_like(t[0])
    pf.poisson_project(plan, *t, phi, gdt, c)
    torch.cuda.synchronize()
    got = [a.cpu().numpy() for a in t] + [phi.cpu().numpy()]
    for name, g, r in zip(("u", "v", "w", "p", "phi"), got, ref):
        check(g, r, TOL[prec], name)
    if prec != "fp32":
        # the projected field is divergence-free with the walls' fluxes
        d1 = oproj.divergence(*got[:3], zf, LX, LY, ogrid.Y_WALLS)
        d0 = oproj.divergence(u, v, w, zf, LX, LY, ogrid.Y_WALLS)
        assert np.sqrt(np.sum(d1 ** 2)) <= TOL[prec] * np.sqrt(np.sum(d0 ** 2))


def test_mixed_y_boundaries_in_one_task_batch():
    """Poisson problems with periodic y, zero-gradient and value-zero y walls
    spread over internal streams give, bitwise, what each gives alone."""
    stream = torch.cuda.Stream(device=_dev())
    specs = [(128, 96, 40, "periodic"), (64, 64, 33, "walls"), (96, 128, 24, "dirichlet"),
             (64, 192, 17, "walls"), (192, 64, 20, "dirichlet"), (64, 96, 48, "periodic")]
    items = []
    for t, (nx, ny, nz, ybc) in enumerate(specs):
        zf = synth.tanh_faces(nz, 2.0, 1.5)
        plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine",
                               stream=stream, ybc=ybc)
        rhs = torch.from_numpy(synth.uniform_pm1(360 + t, (nz, ny, nx))).to(_dev())
        items.append((plan, rhs))
    torch.cuda.synchronize()
    ref = []
    with torch.cuda.stream(stream):
        for plan, rhs in items:
            p = torch.empty_like(rhs)
            pf.poisson_solve(plan, rhs, p)
            ref.append(p)
    stream.synchronize()
    outs = [torch.full_like(rhs, -1.0) for _, rhs in items]
    torch.cuda.synchronize()
    tasks = [dict(poisson=plan, rhs=rhs, p=o) for (plan, rhs), o in zip(items, outs)]
    pf.run_batched(tasks, lanes=4, stream=stream)
    stream.synchronize()
    for t, (o, r) in enumerate(zip(outs, ref)):
        assert torch.equal(o, r), specs[t]
