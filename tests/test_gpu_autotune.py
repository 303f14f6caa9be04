"""Autotuner: every candidate shape computes the same solution, the tuner
keeps the fastest, and the cache round-trips."""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
from paper_2502_06296_amd import autotune
import synth
from oracle import grid as ogrid
from oracle import poisson as op

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32_refine", 1e-10)])
def test_every_zsolve_variant_matches_oracle(prec, tol):
    nx, ny, nz = 128, 64, 200
    f, zf = synth.channel_rhs(31, nx, ny, nz, beta=1.5)
    ref = op.solve_poisson(f, zf, LX, LY)
    dev = torch.device("cuda", 0)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision=prec)
    rhs = torch.from_numpy(f).to(dev)
    p = torch.empty_like(rhs)
    tried = 0
    for v in autotune.zsolve_variants(plan):
        if not autotune.set_zsolve_variant(plan, v):
            continue
        pf.poisson_solve(plan, rhs, p)
        torch.cuda.synchronize()
        err = op.rel_l2(p.cpu().numpy(), ref)
        print(f"variant {v}: {err:.2e}", flush=True)
        assert err < tol, v
        tried += 1
    assert tried >= 4
    times = autotune.tune_poisson(plan, rhs, p, reps=2)
    assert autotune.get_zsolve_variant(plan) == min(times, key=times.get)


def test_pcr_shapes_agree_and_tuner_keeps_fastest(tmp_path):
    nz, ny, nx = 300, 8, 128
    zf = synth.tanh_faces(nz)
    dev = torch.device("cuda", 0)
    al, ga, ex = ogrid.zop(zf, ogrid.DIRICHLET_CENTRE)
    r = synth.normal01(5, (nz, ny, nx))
    ref = op.solve_helmholtz(r, zf, 1e-2, ogrid.DIRICHLET_CENTRE)
    plan = pf.pcr_prepare(al, ga, ex, 1e-2, precision="fp64")
    for m in (8, 16, 32):
        for cw in (16, 32, 64):
            if not autotune.set_pcr_shape([plan], m, cw):
                continue
            u = torch.from_numpy(r).to(dev)
            pf.pcr_apply(plan, u)
            torch.cuda.synchronize()
            assert op.rel_l2(u.cpu().numpy(), ref) < 1e-12, (m, cw)
    u = torch.from_numpy(r).to(dev)
    res = autotune.apply_or_tune_pcr([plan], [u], "fp64", reps=2, path=str(tmp_path / "t.json"))
    assert not res["cached"]
    assert autotune.pcr_shape(plan) == tuple(res["shape"])
    res2 = autotune.apply_or_tune_pcr([plan], [u], "fp64", reps=2, path=str(tmp_path / "t.json"))
    assert res2["cached"] and tuple(res2["shape"]) == tuple(res["shape"])
