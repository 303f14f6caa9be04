"""3-D Helmholtz of a field on the x faces between value-zero walls (the
face-located velocity u of an x-walled grid; the type-I sine transform along
x over the nx - 1 interior faces), alone and with y walls or y faces, through
the C ABI against the CPU oracle, element by element, in the three
precisions; the wall column is zero.

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
YBC = {"periodic": ogrid.Y_PERIODIC, "walls": ogrid.Y_WALLS, "faces": ogrid.Y_FACES}

CASES = [
    (32, 64, 24, 1.5, ogrid.DIRICHLET_CENTRE, 1e-3, 0),    # 64-point transforms
    (96, 96, 20, 2.0, ogrid.DIRICHLET_FACE, 0.05, 1),      # radix-3 (192 points), ragged chunks
    (512, 64, 8, 1.5, ogrid.DIRICHLET_CENTRE, 1e-2, 2),    # 1024-point x transforms
    (1600, 64, 4, 1.2, ogrid.DIRICHLET_CENTRE, 1e-2, 3),   # radix-5 (3200 points)
    (1728, 64, 4, 1.0, ogrid.DIRICHLET_FACE, 1e-2, 4),     # 3456-point x transforms
]


def _run(nx, ny, nz, beta, bc, s, seed, prec, ybc="periodic"):
    zf = synth.tanh_faces(nz, 2.0, beta)
    n = nz if bc == ogrid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(600 + seed, (n, ny, nx))
    ref = op.solve_helmholtz3d(r, zf, s, bc, LX, LY, ybc=YBC[ybc], xbc=ogrid.X_FACES)
    plan = pf.helmholtz3d_plan(nx, ny, nz, H3D_BC[bc], s, LX, LY, 2.0, beta, zf=zf, precision=prec,
                               ybc=ybc, xbc="faces")
    rt = torch.from_numpy(r).to(torch.device("cuda", 0))
    u = torch.full_like(rt, 7.0)
    pf.helmholtz3d_solve(plan, rt, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), ref


@pytest.mark.parametrize("nx,ny,nz,beta,bc,s,seed", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_xfaces_helmholtz3d_matches_oracle(nx, ny, nz, beta, bc, s, seed, prec):
    print(f"helmholtz3d x faces {prec} {nx}x{ny}x{nz} bc={bc} s={s}", flush=True)
    got, ref = _run(nx, ny, nz, beta, bc, s, seed, prec)
    check(got, ref, TOL[prec], prec)
    assert np.max(np.abs(got[:, :, nx - 1])) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("ybc,ny", [("walls", 64), ("faces", 48)])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_xfaces_with_y_walls_or_faces_matches_oracle(ybc, ny, prec):
    print(f"helmholtz3d x faces, y {ybc}, {prec}", flush=True)
    got, ref = _run(96, ny, 24, 1.5, ogrid.DIRICHLET_CENTRE, 2e-2, 7, prec, ybc=ybc)
    check(got, ref, TOL[prec], prec)
    assert np.max(np.abs(got[:, :, 95])) <= 1e-14 * np.max(np.abs(ref))


def test_xfaces_reject_the_poisson_plan():
    with pytest.raises(N.PfError):
        pf.poisson_plan(32, 64, 16, xbc="faces")
