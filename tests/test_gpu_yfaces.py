"""3-D Helmholtz of a field on the y faces between value-zero walls (the
face-located velocity of a y-walled grid; Sec. 2.2.1's sine member, type I,
over the ny - 1 interior faces) through the C ABI against the CPU oracle,
element by element, in the three precisions. The wall row is zero up to the
rounding of the x inverse, which transforms it as the imaginary part of a
line pair with its neighbour row.

Bars: float64 1e-12, float32 with one float64-residual correction 1e-10,
plain float32 1e-5, each for the relative L2 error and for the largest
element-wise error against the largest reference value.
"""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
from paper_2502_06296_amd import _native as N
import synth
from oracle import grid as ogrid
from oracle import poisson as op
from parity import TOL, check

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi
H3D_BC = {ogrid.DIRICHLET_CENTRE: "dirichlet_centre", ogrid.DIRICHLET_FACE: "dirichlet_face"}
XBC = {"periodic": ogrid.X_PERIODIC, "walls": ogrid.X_WALLS, "dirichlet": ogrid.X_DIRICHLET}

CASES = [
    (64, 32, 32, 1.5, ogrid.DIRICHLET_CENTRE, 1e-3, 0),    # 64-point transforms
    (128, 48, 40, 2.0, ogrid.DIRICHLET_FACE, 0.05, 1),     # radix-3 (96 points), ragged chunks
    (96, 1600, 6, 1.2, ogrid.DIRICHLET_CENTRE, 1e-2, 2),   # radix-5 (3200 points)
    (1024, 512, 6, 1.5, ogrid.DIRICHLET_FACE, 1e-3, 3),    # the 1024x512 plane (1024-point y transforms)
    (64, 1728, 4, 1.0, ogrid.DIRICHLET_CENTRE, 1e-2, 4),   # 3456-point y transforms
]


def _run(nx, ny, nz, beta, bc, s, seed, prec, xbc="periodic"):
    zf = synth.tanh_faces(nz, 2.0, beta)
    n = nz if bc == ogrid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(500 + seed, (n, ny, nx))
    ref = op.solve_helmholtz3d(r, zf, s, bc, LX, LY, ybc=ogrid.Y_FACES, xbc=XBC[xbc])
    plan = pf.helmholtz3d_plan(nx, ny, nz, H3D_BC[bc], s, LX, LY, 2.0, beta, zf=zf, precision=prec,
                               ybc="faces", xbc=xbc)
    rt = torch.from_numpy(r).to(torch.device("cuda", 0))
    u = torch.full_like(rt, 7.0)
    pf.helmholtz3d_solve(plan, rt, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), ref


@pytest.mark.parametrize("nx,ny,nz,beta,bc,s,seed", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_yfaces_helmholtz3d_matches_oracle(nx, ny, nz, beta, bc, s, seed, prec):
    print(f"helmholtz3d y faces {prec} {nx}x{ny}x{nz} bc={bc} s={s}", flush=True)
    got, ref = _run(nx, ny, nz, beta, bc, s, seed, prec)
    check(got, ref, TOL[prec], prec)
    assert np.max(np.abs(got[:, ny - 1, :])) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("xbc", ["walls", "dirichlet"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_yfaces_with_x_walls_matches_oracle(xbc, prec):
    print(f"helmholtz3d y faces, x {xbc}, {prec}", flush=True)
    got, ref = _run(128, 48, 24, 1.5, ogrid.DIRICHLET_CENTRE, 2e-2, 7, prec, xbc=xbc)
    check(got, ref, TOL[prec], prec)
    assert np.max(np.abs(got[:, 47, :])) <= 1e-14 * np.max(np.abs(ref))


def test_yfaces_reject_the_poisson_plan():
    with pytest.raises(N.PfError):
        pf.poisson_plan(64, 32, 16, ybc="faces")


def test_yfaces_substeps_captured_in_one_graph():
    """Three Runge-Kutta substeps (a new s each, updated on the device) of the
    face-located field's 3-D Helmholtz, captured in one graph and replayed
    twice: every replay equals the eager run bitwise, and each substep the
    oracle at its own s."""
    nx, ny, nz = 128, 48, 24
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    svals = (2e-2, 5e-3, 1.2e-2)
    plan = pf.helmholtz3d_plan(nx, ny, nz, "dirichlet_centre", svals[0], LX, LY, 2.0, 1.5, zf=zf,
                               precision="fp32_refine", stream=stream, ybc="faces")
    r = [torch.from_numpy(synth.normal01(520 + i, (nz, ny, nx))).to(dev) for i in range(3)]
    ue = [torch.empty_like(x) for x in r]
    ug = [torch.empty_like(x) for x in r]
    torch.cuda.synchronize()

    def substeps(out):
        for i, s in enumerate(svals):
            pf.helmholtz3d_update(plan, s)
            pf.helmholtz3d_solve(plan, r[i], out[i])

    with torch.cuda.stream(stream):
        substeps(ue)
    stream.synchronize()
    for i, s in enumerate(svals):
        ref = op.solve_helmholtz3d(r[i].cpu().numpy(), zf, s, ogrid.DIRICHLET_CENTRE, LX, LY,
                                   ybc=ogrid.Y_FACES)
        check(ue[i].cpu().numpy(), ref, TOL["fp32_refine"], f"substep {i}")
    pf.pf_graph_begin(stream)
    substeps(ug)
    g = pf.pf_graph_end(stream)
    for rep in range(2):
        with torch.cuda.stream(stream):
            for x in ug:
                x.fill_(-1.0)
        g.launch(stream)
        stream.synchronize()
        for i in range(3):
            assert torch.equal(ug[i], ue[i]), (rep, i)
