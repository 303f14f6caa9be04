"""Grouped launches of batches of independent problems: every stage of the
float32+refinement Poisson solves (and 3-D Helmholtz solves) of a batch runs
as one launch per kernel instance, and Helmholtz fields of several problems
share one launch. Each batched result equals the one-by-one result bitwise
and meets the oracle's bars; batches larger than one launch's job table,
mixed with plans that cannot be grouped, and replayed from a graph, too."""
import numpy as np
import pytest
import torch

import paper_2502_06296_amd as pf
import synth
from oracle import grid as ogrid
from oracle import poisson as op
from paper_2502_06296_amd import _native as N
from parity import TOL, check

pytestmark = pytest.mark.gpu
LX, LY = 2 * np.pi, np.pi
S = 0.5 * (1.0 / 5200.0) * 1e-4


def _dev():
    return torch.device("cuda", 0)


def _spec(sp):
    """(nx, ny, nz, beta, precision, kind, ybc) with the defaults filled in."""
    return tuple(sp) + ("fp32_refine", "poisson", "periodic")[len(sp) - 4:]


def _rhs(t, sp):
    nx, ny, nz, beta, prec, kind, ybc = _spec(sp)
    f, zf = synth.channel_rhs(900 + t, nx, ny, nz, beta=beta)
    if kind != "poisson":
        f = synth.normal01(950 + t, (nz, ny, nx))
    return f, zf


def _problem(t, sp, stream=None):
    nx, ny, nz, beta, prec, kind, ybc = _spec(sp)
    f, zf = _rhs(t, sp)
    if kind == "poisson":
        plan = pf.poisson_plan(nx, ny, nz, LX, LY, 2.0, beta, zf=zf, precision=prec, ybc=ybc,
                               stream=stream)
    else:
        plan = pf.helmholtz3d_plan(nx, ny, nz, "dirichlet_centre", 3e-3, LX, LY, 2.0, beta, zf=zf,
                                   precision=prec, ybc=ybc, stream=stream)
    return plan, torch.from_numpy(f).to(_dev())


def _run(specs, check_oracle):
    plans, rhs, outs, singles = [], [], [], []
    for t, sp in enumerate(specs):
        print(f"batch entry {t}: {_spec(sp)}", flush=True)
        plan, r = _problem(t, sp)
        plans.append(plan)
        rhs.append(r)
        outs.append(torch.full_like(r, -1.0))
        singles.append(torch.empty_like(r))
    pf.poisson_solve_batched(plans, rhs, outs)
    for sp, pl, r, s1 in zip(specs, plans, rhs, singles):
        (pf.poisson_solve if _spec(sp)[5] == "poisson" else pf.helmholtz3d_solve)(pl, r, s1)
    torch.cuda.synchronize()
    for t, (a, b) in enumerate(zip(outs, singles)):
        assert torch.equal(a, b), (t, specs[t])
    for t in check_oracle:
        nx, ny, nz, beta, prec, kind, ybc = _spec(specs[t])
        f, zf = _rhs(t, specs[t])
        yb = {"periodic": ogrid.Y_PERIODIC, "walls": ogrid.Y_WALLS}[ybc]
        if kind == "poisson":
            ref = op.solve_poisson(f, zf, LX, LY, ybc=yb)
        else:
            ref = op.solve_helmholtz3d(f, zf, 3e-3, ogrid.DIRICHLET_CENTRE, LX, LY, ybc=yb)
        check(outs[t].cpu().numpy(), ref, TOL[prec], f"entry {t} {_spec(specs[t])}")


def test_uneven_grouped_batch_equals_single_and_oracle():
    shapes = synth.draw_uneven_batch(1, 16)
    specs = [(sh["nx"], sh["ny"], sh["nz"], sh["beta"]) for sh in shapes]
    small = sorted(range(16), key=lambda t: specs[t][0] * specs[t][1] * specs[t][2])[:4]
    _run(specs, small)


def test_mixed_batch_groups_what_it_can():
    """Poisson and 3-D Helmholtz plans of the same lengths share launches;
    a float64 plan and a y-walled plan run after them, one by one."""
    specs = [(64, 64, 40, 1.5), (64, 64, 40, 1.2, "fp32_refine", "helmholtz3d"),
             (128, 64, 40, 1.5), (64, 128, 33, 2.0), (128, 64, 96, 1.0, "fp32_refine", "helmholtz3d"),
             (64, 64, 40, 1.5, "fp64"), (96, 64, 24, 1.5, "fp32_refine", "poisson", "walls"),
             (192, 96, 20, 1.5)]
    _run(specs, range(len(specs)))


def test_grouped_batch_of_long_columns():
    """Columns of more than 512 rows take the 1024-thread z-solve shapes
    (double-buffered reduced rows): still grouped, bitwise equal to the single
    solves, at the oracle."""
    specs = [(64, 64, 600, 1.5), (128, 64, 600, 1.3), (64, 64, 600, 1.2, "fp32_refine", "helmholtz3d"),
             (64, 64, 1000, 1.5)]
    _run(specs, [0, 2, 3])


def test_batch_larger_than_one_launch():
    """20 problems of one shape: two launches per stage (16 + 4 jobs)."""
    specs = [(64, 64, 24, 1.0 + 0.05 * t) for t in range(20)]
    _run(specs, [0, 19])


def test_grouped_batch_graph_replays_equal_eager():
    stream = torch.cuda.Stream(device=_dev())
    specs = [(64, 64, 40, 1.5), (128, 64, 40, 1.3), (64, 128, 96, 1.7), (64, 64, 40, 1.1),
             (64, 64, 40, 1.2, "fp32_refine", "helmholtz3d")]
    plans, rhs = [], []
    for t, sp in enumerate(specs):
        plan, r = _problem(t, sp, stream=stream)
        plans.append(plan)
        rhs.append(r)
    eager = [torch.empty_like(r) for r in rhs]
    outs = [torch.empty_like(r) for r in rhs]
    scratch = torch.empty_like(rhs[0])
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        pf.poisson_solve_batched(plans, rhs, eager)
    stream.synchronize()
    pf.pf_graph_begin(stream)
    pf.poisson_solve_batched(plans, rhs, outs)
    g = pf.pf_graph_end(stream)
    for rep in range(3):
        with torch.cuda.stream(stream):
            for o in outs:
                o.fill_(-1.0)
            pf.poisson_solve(plans[0], rhs[0], scratch)   # eager work between the replays
        g.launch(stream)
        stream.synchronize()
        for t, (o, e) in enumerate(zip(outs, eager)):
            assert torch.equal(o, e), (rep, t)


def test_grouped_batch_records_the_status_of_each_plan():
    specs = [(64, 64, 40, 1.5), (128, 64, 40, 1.3)]
    plans, rhs, sts = [], [], []
    for t, sp in enumerate(specs):
        plan, r = _problem(t, sp)
        st = torch.full((4,), -7, dtype=torch.int64, device=_dev())
        pf.poisson_set_status(plan, st, 1e-10)
        plans.append(plan)
        rhs.append(r)
        sts.append(st)
    outs = [torch.empty_like(r) for r in rhs]
    pf.poisson_solve_batched(plans, rhs, outs)
    torch.cuda.synchronize()
    batched = [s.clone() for s in sts]
    for pl, r, o in zip(plans, rhs, outs):
        pf.poisson_solve(pl, r, o)
    torch.cuda.synchronize()
    for a, b in zip(batched, sts):
        assert torch.equal(a, b)
        assert int(a[3]) == 0


def test_batched_helmholtz_fields_of_several_problems_in_one_launch():
    """12 fields (u, v, w of four problems with one chunk height) in one
    launch equal the fields applied one problem at a time."""
    plans, fields, singles = [], [], []
    nz = 96
    for t in range(4):
        zf = synth.tanh_faces(nz, 2.0, 1.2 + 0.2 * t)
        for c, bc in enumerate((ogrid.DIRICHLET_CENTRE, ogrid.DIRICHLET_CENTRE, ogrid.DIRICHLET_FACE)):
            al, ga, ex = ogrid.zop(zf, bc)
            plans.append(pf.pcr_prepare(al, ga, ex, S * (1 + t), precision="fp32_refine"))
            n = nz if c < 2 else nz - 1
            nx, ny = (64, 64) if t % 2 == 0 else (128, 32)
            f = torch.from_numpy(synth.normal01(970 + 3 * t + c, (n, ny, nx))).to(_dev())
            fields.append(f.clone())
            singles.append(f.clone())
    pf.pcr_apply_batched(plans, fields)
    for pl, f in zip(plans, singles):
        pf.pcr_apply(pl, f)
    torch.cuda.synchronize()
    for a, b in zip(fields, singles):
        assert torch.equal(a, b)


def test_grouped_batch_rejects_shared_plans_and_overlaps():
    p1, r1 = _problem(0, (64, 64, 24, 1.5))
    p2, r2 = _problem(1, (64, 64, 24, 1.5))
    a, b = torch.empty_like(r1), torch.empty_like(r1)
    with pytest.raises(N.PfError) as e:
        pf.poisson_solve_batched([p1, p1], [r1, r2], [a, b])
    assert e.value.code == N.PF_ERR_ARG
    with pytest.raises(N.PfError) as e:      # both write a
        pf.poisson_solve_batched([p1, p2], [r1, r2], [a, a])
    assert e.value.code == N.PF_ERR_ARG
    with pytest.raises(N.PfError) as e:      # the first writes what the second reads
        pf.poisson_solve_batched([p1, p2], [r1, a], [a, b])
    assert e.value.code == N.PF_ERR_ARG



def test_plans_with_tuned_transform_shapes_run_one_by_one():
    from paper_2502_06296_amd import autotune
    specs = [(256, 64, 24, 1.5), (256, 64, 24, 1.3), (256, 64, 24, 1.1)]
    plans, rhs = [], []
    for t, sp in enumerate(specs):
        plan, r = _problem(t, sp)
        plans.append(plan)
        rhs.append(r)
    assert autotune.set_variant(plans[1], autotune.STAGE_XFWD, 3)
    outs = [torch.empty_like(r) for r in rhs]
    singles = [torch.empty_like(r) for r in rhs]
    pf.poisson_solve_batched(plans, rhs, outs)
    for pl, r, s1 in zip(plans, rhs, singles):
        pf.poisson_solve(pl, r, s1)
    torch.cuda.synchronize()
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)
