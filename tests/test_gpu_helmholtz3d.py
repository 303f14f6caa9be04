"""The 3-D implicit Helmholtz (paper Sec. 2.1, eq. proj2_ustar) through the C
ABI against the CPU oracle, element by element, and at the 1024x512x512
channel shape by its float64 residual on the device.

Bars: float64 1e-12, float32 with one float64-residual correction 1e-10,
plain float32 1e-5, each for the relative L2 error and for the largest
element-wise error against the largest reference value.
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
TOL = {"fp64": 1e-12, "fp32_refine": 1e-10, "fp32": 1e-5}
BC = {ogrid.DIRICHLET_CENTRE: "dirichlet_centre", ogrid.DIRICHLET_FACE: "dirichlet_face"}


def _dev():
    return torch.device("cuda", 0)


def _solve_gpu(r, nz, beta, bc, s, prec):
    n, ny, nx = r.shape
    zf = synth.tanh_faces(nz, 2.0, beta)
    plan = pf.helmholtz3d_plan(nx, ny, nz, BC[bc], s, LX, LY, 2.0, beta, zf=zf, precision=prec)
    rt = torch.from_numpy(r).to(_dev())
    u = torch.empty_like(rt)
    pf.helmholtz3d_solve(plan, rt, u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


CASES = [
    (64, 64, 64, 1.5, ogrid.DIRICHLET_CENTRE, 1e-3, 0),
    (64, 64, 64, 1.5, ogrid.DIRICHLET_FACE, 1e-3, 1),
    (128, 96, 40, 2.0, ogrid.DIRICHLET_CENTRE, 0.5, 2),     # strong diffusion, radix-3 y
    (192, 64, 33, 0.0, ogrid.DIRICHLET_FACE, 0.05, 3),      # uniform z, ragged chunks
    (96, 128, 9, 1.2, ogrid.DIRICHLET_CENTRE, 9.615e-9, 4),  # nearly the identity
    (3456, 64, 30, 1.5, ogrid.DIRICHLET_FACE, 1e-3, 5),     # the weak-scaling share's x length
    (3200, 64, 28, 1.5, ogrid.DIRICHLET_CENTRE, 1e-3, 6),   # radix-5 x
    (1024, 512, 8, 1.5, ogrid.DIRICHLET_CENTRE, 9.615e-9, 7),  # the 1024x512x512 workload's lengths
    (2048, 1024, 5, 1.5, ogrid.DIRICHLET_FACE, 1e-3, 8),    # the 2048x1024x1024 workload's lengths
    (256, 64, 512, 1.5, ogrid.DIRICHLET_FACE, 1e-3, 9),     # its z length: the same z-solve shape
]


@pytest.mark.parametrize("nx,ny,nz,beta,bc,s,seed", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_helmholtz3d_matches_oracle(nx, ny, nz, beta, bc, s, seed, prec):
    print(f"helmholtz3d {prec} {nx}x{ny}x{nz} bc={bc} s={s}", flush=True)
    zf = synth.tanh_faces(nz, 2.0, beta)
    n = nz if bc == ogrid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(40 + seed, (n, ny, nx))
    ref = op.solve_helmholtz3d(r, zf, s, bc, LX, LY)
    got = _solve_gpu(r, nz, beta, bc, s, prec)
    check(got, ref, TOL[prec], prec)


def test_helmholtz3d_update_matches_a_fresh_plan():
    nx, ny, nz, beta = 64, 64, 32, 1.5
    zf = synth.tanh_faces(nz, 2.0, beta)
    r = torch.from_numpy(synth.normal01(50, (nz, ny, nx))).to(_dev())
    plan = pf.helmholtz3d_plan(nx, ny, nz, "dirichlet_centre", 0.1, LX, LY, 2.0, beta, precision="fp32_refine")
    pf.helmholtz3d_update(plan, 0.02)
    a = torch.empty_like(r)
    pf.helmholtz3d_solve(plan, r, a)
    fresh = pf.helmholtz3d_plan(nx, ny, nz, "dirichlet_centre", 0.02, LX, LY, 2.0, beta, precision="fp32_refine")
    b = torch.empty_like(r)
    pf.helmholtz3d_solve(fresh, r, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref = op.solve_helmholtz3d(r.cpu().numpy(), zf, 0.02, ogrid.DIRICHLET_CENTRE, LX, LY)
    check(a.cpu().numpy(), ref, 1e-10, "fp32_refine")


def test_plan_kinds_are_not_interchangeable():
    plan = pf.helmholtz3d_plan(64, 64, 16, "dirichlet_centre", 0.1)
    f = torch.zeros((16, 64, 64), dtype=torch.float64, device=_dev())
    with pytest.raises(pf.solver.N.PfError):
        pf.poisson_solve(plan, f, torch.empty_like(f))
    pp = pf.poisson_plan(64, 64, 16)
    with pytest.raises(pf.solver.N.PfError):
        pf.helmholtz3d_solve(pp, f, torch.empty_like(f))


def _residual_dev(u, r, zf, s, bc):
    """||(I - s L) u - r|| / ||r|| in float64 on the device (test-side)."""
    n, ny, nx = u.shape
    al, ga, ex = (torch.from_numpy(np.ascontiguousarray(a)).to(u.device) for a in ogrid.zop(zf, bc))
    rr = nn = 0.0
    for k0 in range(0, n, 64):
        k1 = min(n, k0 + 64)
        c = u[k0:k1]
        lu = (torch.roll(c, -1, 2) - 2 * c + torch.roll(c, 1, 2)) * (nx / LX) ** 2
        lu += (torch.roll(c, -1, 1) - 2 * c + torch.roll(c, 1, 1)) * (ny / LY) ** 2
        lu -= (al + ga + ex)[k0:k1, None, None] * c
        lo = max(k0, 1)
        lu[lo - k0:] += al[lo:k1, None, None] * u[lo - 1:k1 - 1]
        hi = min(k1, n - 1)
        lu[:hi - k0] += ga[k0:hi, None, None] * u[k0 + 1:hi + 1]
        res = c - s * lu - r[k0:k1]
        rr += float(torch.sum(res * res))
        nn += float(torch.sum(r[k0:k1] ** 2))
    return (rr / nn) ** 0.5


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-13), ("fp32_refine", 1e-10)])
def test_helmholtz3d_full_channel_residual(prec, bar):
    nx, ny, nz, beta, s = 1024, 512, 512, 1.5, 1e-4
    print(f"helmholtz3d {prec} {nx}x{ny}x{nz} full size", flush=True)
    zf = synth.tanh_faces(nz, 2.0, beta)
    g = torch.Generator(device=_dev()).manual_seed(8)
    r = torch.randn((nz - 1, ny, nx), dtype=torch.float64, device=_dev(), generator=g)
    plan = pf.helmholtz3d_plan(nx, ny, nz, "dirichlet_face", s, precision=prec)
    u = torch.empty_like(r)
    pf.helmholtz3d_solve(plan, r, u)
    torch.cuda.synchronize()
    res = _residual_dev(u, r, zf, s, ogrid.DIRICHLET_FACE)
    print(f"  residual {res:.2e}", flush=True)
    assert res < bar
