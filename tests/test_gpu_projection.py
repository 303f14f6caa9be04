"""Pressure projection (paper Sec. 2.1, eqs. proj1_Lphi, proj1_ukp1,
proj1_Pkp1, proj2_Pkp1) through the C ABI against the CPU oracle, element by
element; at the full 1024x512x512 channel shape the projected field's
divergence (float64, formed on the device by the test) against the
divergence it started from.

Bars per field: float64 1e-12, float32 with one float64-residual correction
1e-10, plain float32 1e-5, each for the relative L2 error and for the
largest element-wise error against the largest reference value.
"""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
import synth
from oracle import projection as oproj
from oracle import poisson as op
from parity import check

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi
TOL = {"fp64": 1e-12, "fp32_refine": 1e-10, "fp32": 1e-5}


def _dev():
    return torch.device("cuda", 0)


def _inputs(seed, nx, ny, nz):
    u = synth.uniform_pm1(seed, (nz, ny, nx))
    v = synth.uniform_pm1(seed + 1, (nz, ny, nx))
    w = synth.uniform_pm1(seed + 2, (nz - 1, ny, nx))
    p = synth.uniform_pm1(seed + 3, (nz, ny, nx))
    return u, v, w, p


def _project_gpu(u, v, w, p, zf, beta, prec, gdt, c):
    nz, ny, nx = u.shape
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta, zf=zf, precision=prec)
    t = [torch.from_numpy(a).to(_dev()) for a in (u, v, w, p)]
    phi = torch.empty_like(t[0])
    pf.poisson_project(plan, *t, phi, gdt, c)
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in t] + [phi.cpu().numpy()]


PROJ_CASES = [
    (64, 64, 64, 1.5, 0.0, 0),     # the 64^3 channel, explicit diffusion
    (64, 64, 64, 1.5, 1e-3, 1),    # with the implicit z-diffusion pressure term
    (128, 96, 40, 2.0, 0.0, 2),    # radix-3 y, ragged z chunks
    (192, 64, 33, 0.0, 5e-4, 3),   # radix-3 x, uniform z
    (96, 128, 9, 1.2, 0.0, 4),     # few planes; nx not a multiple of the update's 64-column tile
    (3456, 64, 12, 1.5, 1e-3, 5),  # the long x lines: radix-9 divergence pass
    (3200, 96, 9, 1.5, 0.0, 6),    # radix-5 x
    (1024, 512, 8, 1.5, 1e-3, 7),  # the 1024x512x512 workload's x and y lengths
    (2048, 64, 12, 1.5, 0.0, 8),   # the 2048x1024x1024 workload's x length
]


@pytest.mark.parametrize("nx,ny,nz,beta,c,seed", PROJ_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_projection_matches_oracle(nx, ny, nz, beta, c, seed, prec):
    print(f"projection {prec} {nx}x{ny}x{nz} beta={beta} c={c} seed={seed}", flush=True)
    zf = synth.tanh_faces(nz, 2.0, beta)
    u, v, w, p = _inputs(seed, nx, ny, nz)
    gdt = 0.37
    ref = oproj.project(u, v, w, p, zf, LX, LY, gdt, c)
    got = _project_gpu(u, v, w, p, zf, beta, prec, gdt, c)
    for name, g, r in zip(("u", "v", "w", "p", "phi"), got, ref):
        check(g, r, TOL[prec], name)


def test_projection_removes_a_gradient_field():
    nx, ny, nz, beta = 64, 64, 48, 1.5
    zf = synth.tanh_faces(nz, 2.0, beta)
    psi = synth.uniform_pm1(9, (nz, ny, nx))
    u, v, w = oproj.gradient(psi, zf, LX, LY)
    got = _project_gpu(u, v, w, np.zeros_like(u), zf, beta, "fp64", 0.5, 0.0)
    big = max(np.abs(x).max() for x in (u, v, w))
    for x in got[:3]:
        assert np.abs(x).max() <= 1e-11 * big


def _div_dev(u, v, w, zf, lx, ly):
    """Test-side float64 divergence on the device (torch ops)."""
    nz, ny, nx = u.shape
    dzf = torch.from_numpy(np.diff(zf)).to(u.device)
    d = (u - torch.roll(u, 1, dims=2)) * (nx / lx) + (v - torch.roll(v, 1, dims=1)) * (ny / ly)
    d[:-1] += w / dzf[:-1, None, None]
    d[1:] -= w / dzf[1:, None, None]
    return d


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-12), ("fp32_refine", 1e-10)])
def test_projection_full_channel_is_divergence_free(prec, bar):
    nx, ny, nz, beta = 1024, 512, 512, 1.5
    print(f"projection {prec} {nx}x{ny}x{nz} full size", flush=True)
    zf = synth.tanh_faces(nz, 2.0, beta)
    g = torch.Generator(device=_dev()).manual_seed(5)
    u = torch.rand((nz, ny, nx), dtype=torch.float64, device=_dev(), generator=g) * 2 - 1
    v = torch.rand((nz, ny, nx), dtype=torch.float64, device=_dev(), generator=g) * 2 - 1
    w = torch.rand((nz - 1, ny, nx), dtype=torch.float64, device=_dev(), generator=g) * 2 - 1
    p = torch.zeros_like(u)
    d0 = torch.linalg.vector_norm(_div_dev(u, v, w, zf, LX, LY)).item()
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta, precision=prec)
    phi = torch.empty_like(u)
    pf.poisson_project(plan, u, v, w, p, phi, 0.25, 0.0)
    torch.cuda.synchronize()
    d1 = torch.linalg.vector_norm(_div_dev(u, v, w, zf, LX, LY)).item()
    print(f"  |D u| before {d0:.3e} after {d1:.3e} ratio {d1 / d0:.3e}", flush=True)
    assert d1 <= bar * d0
    # p += phi with c = 0
    assert torch.equal(p, phi)
