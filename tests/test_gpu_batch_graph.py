"""Batched and graph-captured execution (the uneven batch and the captured
projection step): batched results equal one-by-one results bitwise, every
graph replay equals the eager result bitwise, and the batch meets the
oracle's bar."""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
import synth
from oracle import grid as ogrid
from oracle import poisson as op

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi
S = 0.5 * (1.0 / 5200.0) * 1e-4


def _dev():
    return torch.device("cuda", 0)


def test_uneven_batch_matches_single_and_oracle():
    shapes = synth.draw_uneven_batch(0, 16)
    plans, rhs, outs, singles, refs = [], [], [], [], []
    for t, sh in enumerate(shapes):
        nx, ny, nz, beta = sh["nx"], sh["ny"], sh["nz"], sh["beta"]
        print(f"batch item {t}: {nx}x{ny}x{nz} beta={beta:.3f}", flush=True)
        f, zf = synth.channel_rhs(100 + t, nx, ny, nz, beta=beta)
        plans.append(pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta, zf=zf, precision="fp32_refine"))
        r = torch.from_numpy(f).to(_dev())
        rhs.append(r)
        outs.append(torch.empty_like(r))
        singles.append(torch.empty_like(r))
        if t < 4:
            refs.append(op.solve_poisson(f, zf, LX, LY))
    pf.poisson_solve_batched(plans, rhs, outs)
    for pl, r, s1 in zip(plans, rhs, singles):
        pf.poisson_solve(pl, r, s1)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)
    for ref, got in zip(refs, outs):
        assert op.rel_l2(got.cpu().numpy(), ref) < 1e-10


def _projection_setup(prec, nx=128, ny=64, nz=96, beta=1.5):
    f, zf = synth.channel_rhs(7, nx, ny, nz, beta=beta)
    stream = torch.cuda.Stream(device=_dev())
    with torch.cuda.stream(stream):
        pp = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta, zf=zf, precision=prec, stream=stream)
        pcr = []
        for bc in (ogrid.DIRICHLET_CENTRE, ogrid.DIRICHLET_CENTRE, ogrid.DIRICHLET_FACE):
            al, ga, ex = ogrid.zop(zf, bc)
            pcr.append(pf.pcr_prepare(al, ga, ex, S, precision=prec, stream=stream))
        rhs = torch.from_numpy(f).to(_dev())
        r3 = [torch.from_numpy(synth.normal01(20 + c, (nz if c < 2 else nz - 1, ny, nx))).to(_dev())
              for c in range(3)]
    return pp, pcr, rhs, r3, stream


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_graph_replay_equals_eager(prec):
    pp, pcr, rhs, r3, stream = _projection_setup(prec)
    u = [r.clone() for r in r3]
    p = torch.empty_like(rhs)
    # eager reference
    ue = [r.clone() for r in r3]
    pe = torch.empty_like(rhs)
    with torch.cuda.stream(stream):
        pf.pcr_apply_batched(pcr, ue)
        pf.poisson_solve(pp, rhs, pe)
    stream.synchronize()
    # capture
    pf.pf_graph_begin(stream)
    pf.pcr_apply_batched(pcr, u)
    pf.poisson_solve(pp, rhs, p)
    g = pf.pf_graph_end(stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            for a, b in zip(u, r3):
                a.copy_(b)                # eager work between the replays
            p.fill_(-1.0)
        g.launch(stream)
        stream.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(p, pe), rep
        for a, b in zip(u, ue):
            assert torch.equal(a, b), rep
