"""The a-posteriori status of the float32 refinement (the device flag of the
refinement control): a normal solve records a small estimate and no flag;
a zero tolerance forces the flag from the host; solves without a correction
record -1; graph replays rewrite it (its reset is a kernel, not a memset)."""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
import synth
from oracle import poisson as op

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi


def _dev():
    return torch.device("cuda", 0)


def _setup(prec, tol, nx=128, ny=64, nz=96):
    f, zf = synth.channel_rhs(5, nx, ny, nz, beta=1.5)
    plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, 1.5, zf=zf, precision=prec)
    st = torch.full((4,), -7, dtype=torch.int64, device=_dev())
    pf.poisson_set_status(plan, st, tol)
    rhs = torch.from_numpy(f).to(_dev())
    return plan, st, rhs, f, zf


def test_refined_solve_records_a_small_estimate():
    plan, st, rhs, f, zf = _setup("fp32_refine", 1e-10)
    p = torch.empty_like(rhs)
    pf.poisson_solve(plan, rhs, p)
    torch.cuda.synchronize()
    est, flags = pf.read_status(st)
    err = op.rel_l2(p.cpu().numpy(), op.solve_poisson(f, zf, LX, LY))
    print(f"estimate {est:.2e}, error against the oracle {err:.2e}", flush=True)
    assert 0.0 < est < 1e-10 and flags == 0
    assert err < 1e-10


def test_zero_tolerance_raises_the_flag():
    plan, st, rhs, _, _ = _setup("fp32_refine", 0.0)
    p = torch.empty_like(rhs)
    pf.poisson_solve(plan, rhs, p)
    torch.cuda.synchronize()
    est, flags = pf.read_status(st)
    assert est > 0.0 and flags == 1


def test_unrefined_solves_record_minus_one():
    for prec in ("fp64", "fp32"):
        plan, st, rhs, _, _ = _setup(prec, 1e-10)
        p = torch.empty_like(rhs)
        pf.poisson_solve(plan, rhs, p)
        torch.cuda.synchronize()
        assert pf.read_status(st) == (-1.0, 0)


def test_status_in_graph_replays():
    stream = torch.cuda.Stream(device=_dev())
    f, zf = synth.channel_rhs(6, 128, 64, 48, beta=1.5)
    with torch.cuda.stream(stream):
        plan = pf.poisson_plan(128, 64, 48, LX, LY, 2.0, 1.5, zf=zf, precision="fp32_refine", stream=stream)
        st = torch.zeros(4, dtype=torch.int64, device=_dev())
        rhs = torch.from_numpy(f).to(_dev())
        p = torch.empty_like(rhs)
    stream.synchronize()
    pf.poisson_set_status(plan, st, 1e-10)
    with torch.cuda.stream(stream):
        pf.poisson_solve(plan, rhs, p)
    stream.synchronize()
    eager = pf.read_status(st)
    pf.pf_graph_begin(stream)
    pf.poisson_solve(plan, rhs, p)
    g = pf.pf_graph_end(stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            st.fill_(123)                 # eager work between the replays
        g.launch(stream)
        stream.synchronize()
        assert pf.read_status(st) == eager, rep
