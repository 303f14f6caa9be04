"""Invariants of the HIP path that hold whatever the oracle says: run-to-run
bitwise repeatability (no atomics or unordered reductions in the data
path), translation invariance in the periodic directions and linearity."""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
import synth
from oracle import poisson as op

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi
TOL = {"fp64": 1e-12, "fp32_refine": 1e-10, "fp32": 1e-5}


def _dev():
    return torch.device("cuda", 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_run_to_run_bitwise(prec):
    nx, ny, nz = 128, 96, 72
    f, zf = synth.channel_rhs(21, nx, ny, nz, beta=1.5)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision=prec)
    rhs = torch.from_numpy(f).to(_dev())
    a, b = torch.empty_like(rhs), torch.empty_like(rhs)
    pf.poisson_solve(plan, rhs, a)
    pf.poisson_solve(plan, rhs, b)
    r = torch.from_numpy(synth.normal01(22, (nz, ny, nx))).to(_dev(), torch.float32 if prec == "fp32" else torch.float64)
    al, ga, ex = pf.zop_rows(nz, "dirichlet_centre", 2.0, 1.5)
    hp = pf.pcr_prepare(al, ga, ex, 1e-3, precision=prec)
    u1, u2 = r.clone(), r.clone()
    pf.pcr_apply(hp, u1)
    pf.pcr_apply(hp, u2)
    h3 = pf.helmholtz3d_plan(nx, ny, nz, "dirichlet_centre", 1e-3, LX, LY, 2.0, 1.5, precision=prec)
    r64 = r.double()
    v1, v2 = torch.empty_like(r64), torch.empty_like(r64)
    pf.helmholtz3d_solve(h3, r64, v1)
    pf.helmholtz3d_solve(h3, r64, v2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(u1, u2)
    assert torch.equal(v1, v2)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_translation_invariance_and_linearity(prec):
    nx, ny, nz = 128, 64, 40
    f, zf = synth.channel_rhs(23, nx, ny, nz, beta=1.5)
    g, _ = synth.channel_rhs(24, nx, ny, nz, beta=1.5)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision=prec)

    def solve(x):
        t = torch.from_numpy(np.ascontiguousarray(x)).to(_dev())
        p = torch.empty_like(t)
        pf.poisson_solve(plan, t, p)
        torch.cuda.synchronize()
        return p.cpu().numpy()

    pf_ = solve(f)
    shifted = solve(np.roll(np.roll(f, 5, axis=2), -3, axis=1))
    assert op.rel_l2(shifted, np.roll(np.roll(pf_, 5, axis=2), -3, axis=1)) < TOL[prec]
    pg = solve(g)
    comb = solve(0.75 * f - 2.5 * g)
    assert op.rel_l2(comb, 0.75 * pf_ - 2.5 * pg) < TOL[prec]


@pytest.mark.parametrize("nbytes", [16, 16 * 1023, 16 * 1024, 16 * 1024 * 37 + 16 * 5, (64 << 20) + 48])
def test_calibration_copy_copies_every_byte(nbytes):
    """The byte-counter calibration copy: whole 16 KiB tiles plus a ragged
    tail, every byte copied and nothing past the end written."""
    g = torch.Generator(device="cpu").manual_seed(nbytes % 1000)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).to(_dev())
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device=_dev())
    pf.pf_copy_kernel(dst[:nbytes], src)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert torch.all(dst[nbytes:] == 0)
