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


@pytest.mark.parametrize("xbc", ["walls", "dirichlet"])
def test_every_zsolve_variant_matches_oracle_with_x_walls(xbc):
    # x walls: every column pair carries two shifts, so each variant's
    # two-pass path runs on every tile
    nx, ny, nz = 128, 64, 120
    f, zf = synth.channel_rhs(37, nx, ny, nz, beta=1.5)
    xc = {"walls": ogrid.X_WALLS, "dirichlet": ogrid.X_DIRICHLET}[xbc]
    ref = op.solve_poisson(f, zf, LX, LY, xbc=xc)
    dev = torch.device("cuda", 0)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine", xbc=xbc)
    rhs = torch.from_numpy(f).to(dev)
    p = torch.empty_like(rhs)
    tried = 0
    for v in autotune.zsolve_variants(plan):
        if not autotune.set_zsolve_variant(plan, v):
            continue
        pf.poisson_solve(plan, rhs, p)
        torch.cuda.synchronize()
        err = op.rel_l2(p.cpu().numpy(), ref)
        print(f"x {xbc} variant {v}: {err:.2e}", flush=True)
        assert err < 1e-10, v
        tried += 1
    assert tried >= 4


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


TSHAPES = [(256, 512, 24, 3), (1024, 256, 12, 4), (2048, 64, 8, 5), (512, 1024, 8, 6), (64, 3072, 4, 7),
           (96, 3456, 4, 8), (128, 3200, 4, 9)]


@pytest.mark.parametrize("nx,ny,nz,seed", TSHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine", "fp32"])
def test_every_transform_shape_matches_oracle(nx, ny, nz, seed, prec):
    """The launch shapes of each periodic direction (threads per line, lines
    per workgroup, radix at most 8, the persistent y transforms) meet the
    oracle's bar; with float32 storage shapes 1, 2 and 4 give the default's
    result bitwise (the butterflies are the same; only the compiler's fusion
    of their multiply-adds may differ, below float32 rounding)."""
    from parity import TOL, check
    print(f"transform shapes {prec} {nx}x{ny}x{nz}", flush=True)
    f, zf = synth.channel_rhs(40 + seed, nx, ny, nz, beta=1.5)
    ref = op.solve_poisson(f, zf, LX, LY)
    dev = torch.device("cuda", 0)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision=prec, tuned=False)
    rhs = torch.from_numpy(f).to(dev)
    p0 = torch.empty_like(rhs)
    pf.poisson_solve(plan, rhs, p0)
    torch.cuda.synchronize()
    tried = 0
    for stage in (autotune.STAGE_XFWD, autotune.STAGE_YFWD):
        for v in range(autotune.transform_shape_count(plan)):
            if not autotune.set_variant(plan, stage, v):
                continue
            p = torch.empty_like(rhs)
            pf.poisson_solve(plan, rhs, p)
            torch.cuda.synchronize()
            if v in (1, 2, 4) and prec == "fp32":
                assert torch.equal(p, p0), (stage, v)
            check(p.cpu().numpy(), ref, TOL[prec], f"stage {stage} shape {v}")
            tried += 1
        autotune.set_variant(plan, stage, 0)
    assert tried >= 2


def test_transform_tuner_caches_and_plans_apply_the_cache(tmp_path, monkeypatch):
    nx, ny, nz = 512, 256, 16
    f, zf = synth.channel_rhs(47, nx, ny, nz, beta=1.5)
    dev = torch.device("cuda", 0)
    path = str(tmp_path / "tune.json")
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine", tuned=False)
    rhs = torch.from_numpy(f).to(dev)
    p = torch.empty_like(rhs)
    res = autotune.apply_or_tune_poisson(plan, rhs, p, "fp32_refine", reps=2, path=path)
    assert not res["cached"]
    tx, ty = res["transform_ms"]["x"], res["transform_ms"]["y"]
    assert autotune.get_variant(plan, autotune.STAGE_XFWD) == min(tx, key=tx.get)
    assert autotune.get_variant(plan, autotune.STAGE_YFWD) == min(ty, key=ty.get)
    monkeypatch.setenv("PF_TUNE_CACHE", path)
    fresh = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine")
    for st in (autotune.STAGE_ZSOLVE, autotune.STAGE_XFWD, autotune.STAGE_YFWD):
        assert autotune.get_variant(fresh, st) == autotune.get_variant(plan, st)
    # a tuned plan and a default one agree within the bar
    q = torch.empty_like(rhs)
    pf.poisson_solve(fresh, rhs, q)
    d = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine", tuned=False)
    r = torch.empty_like(rhs)
    pf.poisson_solve(d, rhs, r)
    torch.cuda.synchronize()
    assert op.rel_l2(q.cpu().numpy(), r.cpu().numpy()) < 1e-10


@pytest.mark.parametrize("nx,ny,nz,yshape,zvar", [(256, 512, 24, 4, 39), (128, 3072, 4, 4, 38),
                                                   (64, 256, 640, 3, 37)])
def test_tuned_shapes_replay_in_a_graph(nx, ny, nz, yshape, zvar):
    """A plan with non-default shapes (the persistent y transforms, whose
    grid comes from an occupancy query; the double-buffered z solves)
    captured in a graph: three replays, with eager work between them, equal
    the eager solve bitwise."""
    from paper_2502_06296_amd import solver
    f, zf = synth.channel_rhs(48, nx, ny, nz, beta=1.5)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine", tuned=False,
                           stream=stream)
    assert autotune.set_variant(plan, autotune.STAGE_YFWD, yshape)
    if not autotune.set_zsolve_variant(plan, zvar):
        pytest.skip(f"z-solve variant {zvar} does not fit {nx}x{ny}x{nz}")
    rhs = torch.from_numpy(f).to(dev)
    pe, pg = torch.empty_like(rhs), torch.empty_like(rhs)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        pf.poisson_solve(plan, rhs, pe)
    stream.synchronize()
    check_ref = op.solve_poisson(f, zf, LX, LY)
    assert op.rel_l2(pe.cpu().numpy(), check_ref) < 1e-10
    pf.pf_graph_begin(stream)
    pf.poisson_solve(plan, rhs, pg)
    g = pf.pf_graph_end(stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            pg.fill_(-1.0)
            pf.poisson_solve(plan, rhs, torch.empty_like(rhs))  # eager work between the replays
        g.launch(stream)
        stream.synchronize()
        assert torch.equal(pg, pe), rep
