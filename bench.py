"""Benchmark of the pressure-projection hot path on one MI355X.

Default workload: one projection step on the 2048 x 1024 x 1024 channel grid
(Lx = 2 pi, Ly = pi, Lz = 2, tanh stretching 1.5; 2^31 points): the
z-implicit Helmholtz solves of the three velocity components (u, v at cell
centres, w at interior faces; one batched launch) followed by the pressure
Poisson solve, inputs resident in HBM (seeded draws on the device:
uniform[-1, 1] with the mean removed for the pressure right-hand side, N(0,1)
for the velocity components). The headline path computes in float32 with one
float64-residual correction (relative error <= 1e-10); the plain float64 path
is timed beside it. The three-component Helmholtz of the 1024 x 1024 x 512
grid is timed in the same run.

Prints one JSON line. Per-kernel times come from HIP events recorded on the
solver's stream around every kernel of the timed steps; the roofline entry
prices the kernel with the largest share of the step against 8 TB/s.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
    python bench.py --workload channel      (1024 x 512 x 512, with the coupled
                                             substep and the 3-D Helmholtz)
    python bench.py --copy-calibration 4294967296   (byte-counter calibration)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the step's grid; set per workload by main()
NX, NY, NZ, BETA = 2048, 1024, 1024, 1.5
SHAPES = {"projection": (2048, 1024, 1024), "channel": (1024, 512, 512)}
HELM_C3 = (1024, 1024, 512)     # the three-component Helmholtz grid
LX, LY, LZ = 2 * math.pi, math.pi, 2.0
S_HELM = 0.5 * (1.0 / 5200.0) * 1e-4     # alpha * nu * dt, Re_tau = 5200
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SOURCES = ["paper_2502_06296_amd/csrc/kernels_fft.hip", "paper_2502_06296_amd/csrc/kernels_fft_alt.hip",
                  "paper_2502_06296_amd/csrc/kernels_fft_pf.hip", "paper_2502_06296_amd/csrc/kernels_z.hip",
                  "paper_2502_06296_amd/csrc/fft_kernels.hpp", "paper_2502_06296_amd/csrc/fft_lds.hpp",
                  "paper_2502_06296_amd/csrc/pf_internal.hpp"]

# algorithmic HBM bytes per grid point of one launch of each stage (one read
# and one write of what the stage must touch; stencil neighbours not counted)
BYTES_PER_POINT = {
    "fp32_refine": {"xfwd": 8 + 4, "yfwd": 8, "zsolve": 8, "yinv": 8,
                    "xfwd_resid": 8 + 4 + 4, "xinv_final": 4 + 4 + 8, "zero_mode": 0,
                    "pcr_apply": 16},
    "fp64": {"xfwd": 16, "yfwd": 16, "zsolve": 16, "yinv": 16, "xinv": 16, "zero_mode": 0,
             "pcr_apply": 16},
}


# the coupled step (divergence right-hand side, projection correction): the
# first x pass reads u, v, w instead of f (and, refined, stashes f for the
# residual); the correction reads phi, u, v, w, p and writes u, v, w, p
COUPLED_BYTES = {
    "fp32_refine": {"xfwd": 24 + 4 + 8, "project": 8 + 32 + 32},
    "fp64": {"xfwd": 24 + 8, "project": 8 + 32 + 32},
}
GDT = 1e-4                      # gamma_k * dt of the projection
C_IMPL = S_HELM                 # gamma_k * nu * dt / 2: implicit z diffusion


def sources_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


HELM_SEED = 11                  # seeds of the velocity components: 11, 12, 13
RHS_SEED = 7


def device_rhs(torch, dev, shape, seed=RHS_SEED):
    """uniform[-1, 1] from a seeded device generator, mean removed (the solve
    removes the dzf-weighted mean itself)."""
    g = torch.Generator(device=dev).manual_seed(seed)
    f = torch.empty(shape, dtype=torch.float64, device=dev)
    f.uniform_(-1.0, 1.0, generator=g)
    f -= f.mean()
    return f


def fill_normal(torch, t, seed):
    g = torch.Generator(device=t.device).manual_seed(seed)
    t.normal_(generator=g)


class Step:
    """Plans and fields of one projection step at one precision: the
    velocity components are N(0, 1) draws of fixed seeds, redrawn by
    reset_fields()."""

    def __init__(self, pf, torch, dev, prec, f, tune=False):
        self.pf, self.torch, self.prec = pf, torch, prec
        self.stream = torch.cuda.Stream(device=dev)
        self.tuned = None
        with torch.cuda.stream(self.stream):
            self.poisson = pf.poisson_plan(NX, NY, NZ, LX, LY, LZ, BETA, precision=prec, n_refine=1,
                                           stream=self.stream, device=dev, tuned=False)
            self.pcr = []
            for bc in ("dirichlet_centre", "dirichlet_centre", "dirichlet_face"):
                al, ga, ex = pf.zop_rows(NZ, bc, LZ, BETA)
                self.pcr.append(pf.pcr_prepare(al, ga, ex, S_HELM, precision=prec, stream=self.stream))
            self.rhs = f
            self.p = torch.empty_like(f)
            self.u = [torch.empty((NZ if c < 2 else NZ - 1, NY, NX), dtype=torch.float64, device=dev)
                      for c in range(3)]
        self.reset_fields()
        if tune:
            # the autotuner's choice of z-solve shape and transform shapes for
            # this grid, timed on the plan's own buffers (a cache in the
            # temporary directory keeps it between runs on one machine)
            from paper_2502_06296_amd import autotune
            with torch.cuda.stream(self.stream):
                res = autotune.apply_or_tune_poisson(self.poisson, f, self.p, prec, reps=2, path=TUNE_CACHE)
            self.stream.synchronize()
            self.tuned = {k: res[k] for k in ("zsolve_variant", "xshape", "yshape", "cached")}

    def reset_fields(self):
        with self.torch.cuda.stream(self.stream):
            for c, u in enumerate(self.u):
                fill_normal(self.torch, u, HELM_SEED + c)

    def run(self):
        self.pf.pcr_apply_batched(self.pcr, self.u)
        self.pf.poisson_solve(self.poisson, self.rhs, self.p)

    def timing(self, on):
        self.pf.poisson_timing(self.poisson, on)
        self.pf.pcr_timing(self.pcr[0], on)

    def read_timing(self):
        t = self.pf.poisson_timing_read(self.poisson)
        t.update(self.pf.pcr_timing_read(self.pcr[0]))
        return t


class CoupledStep:
    """One Runge-Kutta substep's implicit part on real fields: the three
    z-implicit Helmholtz solves of (u, v, w) (u, v on the x and y faces at
    cell-centre heights, w on the interior z faces), then the pressure
    projection of the result (divergence right-hand side, Poisson solve,
    face-gradient correction, pressure update with the implicit-diffusion
    term)."""

    def __init__(self, pf, torch, dev, prec):
        self.pf, self.torch, self.prec = pf, torch, prec
        self.stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(self.stream):
            self.poisson = pf.poisson_plan(NX, NY, NZ, LX, LY, LZ, BETA, precision=prec, n_refine=1,
                                           stream=self.stream, device=dev)
            self.pcr = []
            for bc in ("dirichlet_centre", "dirichlet_centre", "dirichlet_face"):
                al, ga, ex = pf.zop_rows(NZ, bc, LZ, BETA)
                self.pcr.append(pf.pcr_prepare(al, ga, ex, S_HELM, precision=prec, stream=self.stream))
            self.vel = [torch.empty((NZ if c < 2 else NZ - 1, NY, NX), dtype=torch.float64, device=dev)
                        for c in range(3)]
            for c, v in enumerate(self.vel):
                fill_normal(torch, v, HELM_SEED + c)
            self.p = torch.zeros_like(self.vel[0])
            self.phi = torch.empty_like(self.vel[0])

    def run(self):
        self.pf.pcr_apply_batched(self.pcr, self.vel)
        self.pf.poisson_project(self.poisson, *self.vel, self.p, self.phi, GDT, C_IMPL)

    timing = Step.timing
    read_timing = Step.read_timing


def time_steps(step, steps, warmup):
    torch = step.torch
    for _ in range(warmup):
        step.run()
    step.stream.synchronize()
    step.read_timing()                       # discard anything recorded so far
    step.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(step.stream)
    for _ in range(steps):
        step.run()
    end.record(step.stream)
    step.stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = step.read_timing()
    step.timing(False)
    ms = start.elapsed_time(end) / steps
    return ms, wall, stages


def graph_ms(step, reps):
    """Mean ms of the step replayed from one captured HIP graph."""
    pf, torch = step.pf, step.torch
    step.stream.synchronize()
    pf.pf_graph_begin(step.stream)
    step.run()
    g = pf.pf_graph_end(step.stream)
    g.launch(step.stream)
    step.stream.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(step.stream)
    for _ in range(reps):
        g.launch(step.stream)
    b.record(step.stream)
    step.stream.synchronize()
    return a.elapsed_time(b) / reps


def stage_points(stage):
    # pcr_apply covers u, v (nz rows) and w (nz-1 rows) in one launch
    if stage == "pcr_apply":
        return NX * NY * (2 * NZ + NZ - 1)
    return NX * NY * NZ


def traffic_file():
    return os.path.join(ROOT, "profiles", f"traffic_counters_{NX}x{NY}x{NZ}.json")


def roofline(prec, stages, traffic):
    per = BYTES_PER_POINT[prec]
    best = max((s for s in stages if per.get(s, 0) > 0), key=lambda s: stages[s][0])
    ms, n = stages[best]
    avg_ms = ms / n
    algo = per[best] * stage_points(best)
    achieved = algo / (avg_ms * 1e-3) / 1e9
    tr = None
    if traffic and traffic.get("sources") == sources_hash() and traffic.get("shape") == [NX, NY, NZ]:
        entry = traffic.get("kernels", {}).get(f"{prec}:{best}")
        if entry:
            tr = entry["bytes_per_launch"]
    return {"kernel": best, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
            "algorithmic_bytes_per_launch": algo, "avg_launch_ms": round(avg_ms, 4)}


# the oracle's sample of the workload: its z grid on a reduced plane, two
# samples per worker process
CPU_PLANE = (512, 256)
CPU_SAMPLES_PER_WORKER = 1


def _oracle_sample(args):
    """Samples run in one worker process: the float64 oracle's Poisson solve
    and three Helmholtz solves per sample, timed around the solves only
    (returns the summed solve time and the first solve's start)."""
    worker, count, nx, ny, nz = args
    import synth
    from oracle import grid as og
    from oracle import poisson as op
    busy, start = 0.0, None
    for k in range(count):
        seed = worker * count + k
        f, zf = synth.channel_rhs(seed, nx, ny, nz, beta=BETA)
        r = [synth.normal01(1000 + 3 * seed + c, (nz if c < 2 else nz - 1, ny, nx)) for c in range(3)]
        t0 = time.perf_counter()
        start = t0 if start is None else start
        op.solve_poisson(f, zf, LX, LY)
        for c in range(3):
            op.solve_helmholtz(r[c], zf, S_HELM, og.DIRICHLET_CENTRE if c < 2 else og.DIRICHLET_FACE)
        busy += time.perf_counter() - t0
        del f, r
    return busy, start


def host_workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(nz):
    """The float64 oracle (numpy, as written) on a bounded sample of the
    workload, on the host's cores: one sample per worker process (the
    Poisson solve plus the three Helmholtz solves on a 512 x 256 plane with
    the workload's z grid and stretching), all workers at once; the rate is
    the sampled points over the span from the first solve's start to the
    last worker's end (input generation between a worker's two samples
    included). Runs before the GPU is touched (the workers are forked)."""
    import multiprocessing as mp
    nx, ny = CPU_PLANE
    workers, per = host_workers(), CPU_SAMPLES_PER_WORKER
    ctx = mp.get_context("fork")
    t_begin = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_sample, [(w, per, nx, ny, nz) for w in range(workers)])
    t_end = time.perf_counter()
    span = t_end - min(t0 for _, t0 in res)
    pts = nx * ny * nz * workers * per
    return {"value": round(pts / span / 1e9, 6), "unit": "Gpoints/s", "cores": workers, "kind": "oracle",
            "sample": f"float64 numpy oracle, Poisson + 3 Helmholtz on {nx}x{ny}x{nz} (the workload's z "
                      f"grid, tanh {BETA}), {per} seeded samples per worker process, {workers} processes "
                      f"at once, {span:.1f} s span (pool start {t_end - t_begin - span:.1f} s excluded)",
            "seconds": round(span, 2), "cpu_seconds": round(sum(dt for dt, _ in res), 2),
            "host_cpus": os.cpu_count()}


def copy_calibration(nbytes):
    import torch
    import paper_2502_06296_amd as pf
    dev = torch.device("cuda", 0)
    a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        pf.pf_copy_kernel(b, a)
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(10):
        pf.pf_copy_kernel(b, a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / 10
    print(json.dumps({"copy_bytes": nbytes, "ms": ms, "GBps": 2 * nbytes / ms / 1e6}))


def ywalls(args):
    """Poisson alone on the 1024x512x512 grid, periodic in y, with
    zero-gradient y walls (cosine transform along y) and with value-zero y
    walls (sine transform), FP64 and FP32+refine."""
    import torch
    import paper_2502_06296_amd as pf
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    g = torch.Generator(device=dev).manual_seed(4)
    f = torch.rand((NZ, NY, NX), dtype=torch.float64, device=dev, generator=g) * 2 - 1
    f -= f.mean()
    p = torch.empty_like(f)
    npts = NX * NY * NZ
    out = {"workload": f"pressure Poisson alone, {NX}x{NY}x{NZ}, tanh {BETA}: y periodic, zero-gradient "
                       "y walls, value-zero y walls",
           "metric": "Gpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup}
    st = torch.cuda.Stream(device=dev)
    for ybc in ("periodic", "walls", "dirichlet"):
        for prec in ("fp32_refine", "fp64"):
            log(f"ywalls: {ybc} {prec}")
            plan = pf.poisson_plan(NX, NY, NZ, beta=BETA, precision=prec, stream=st, ybc=ybc)
            with torch.cuda.stream(st):
                for _ in range(args.warmup):
                    pf.poisson_solve(plan, f, p)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(st)
                for _ in range(args.steps):
                    pf.poisson_solve(plan, f, p)
                b.record(st)
            b.synchronize()
            ms = a.elapsed_time(b) / args.steps
            out[f"{ybc}_{prec}"] = {"ms_per_solve": round(ms, 4), "gpoints_per_s": round(npts / ms / 1e6, 3)}
            del plan
    print(json.dumps(out), flush=True)


def uneven_batch(args):
    """16 independent problems of uneven sizes (64-256 x 64-256 x 96-384, tanh
    stretching drawn per problem), each a pressure Poisson solve and the
    three Helmholtz fields, FP32+refine, run as one task batch on 1, 2, 4
    and 8 internal streams, eager and replayed from one captured graph."""
    import torch
    import paper_2502_06296_amd as pf
    import synth
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    shapes = synth.draw_uneven_batch(0, 16)
    stream = torch.cuda.Stream(device=dev)
    tasks, pts = [], 0
    with torch.cuda.stream(stream):
        for t, sh in enumerate(shapes):
            nx, ny, nz, beta = sh["nx"], sh["ny"], sh["nz"], sh["beta"]
            pts += nx * ny * nz
            pp = pf.poisson_plan(nx, ny, nz, LX, LY, LZ, beta, precision="fp32_refine", stream=stream,
                                 device=dev)
            g = torch.Generator(device=dev).manual_seed(t)
            f = torch.rand((nz, ny, nx), generator=g, dtype=torch.float64, device=dev)
            pcr, fl = [], []
            for c, bc in enumerate(("dirichlet_centre", "dirichlet_centre", "dirichlet_face")):
                al, ga, ex = pf.zop_rows(nz, bc, LZ, beta)
                pcr.append(pf.pcr_prepare(al, ga, ex, S_HELM, precision="fp32_refine", stream=stream))
                fl.append(torch.randn((nz if c < 2 else nz - 1, ny, nx), generator=g, dtype=torch.float64,
                                      device=dev))
            tasks.append(dict(poisson=pp, rhs=f, p=torch.empty_like(f), pcr=pcr, fields=fl))
    stream.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = []
    for lanes in (1, 2, 4, 8):
        log(f"bench: uneven batch, task batch on {lanes} lanes")
        for _ in range(args.warmup):
            pf.run_batched(tasks, lanes=lanes, stream=stream)
        stream.synchronize()
        a.record(stream)
        for _ in range(args.steps):
            pf.run_batched(tasks, lanes=lanes, stream=stream)
        b.record(stream)
        stream.synchronize()
        ms = a.elapsed_time(b) / args.steps
        pf.pf_graph_begin(stream)
        pf.run_batched(tasks, lanes=lanes, stream=stream)
        gr = pf.pf_graph_end(stream)
        gr.launch(stream)
        stream.synchronize()
        a.record(stream)
        for _ in range(args.steps):
            gr.launch(stream)
        b.record(stream)
        stream.synchronize()
        gms = a.elapsed_time(b) / args.steps
        rows.append({"lanes": lanes, "ms": round(ms, 3), "graph_ms": round(gms, 3),
                     "gpoints_per_s": round(pts / ms / 1e6, 2), "graph_gpoints_per_s": round(pts / gms / 1e6, 2)})
    # grouped launches on the caller's stream: the 48 Helmholtz fields in
    # launches of up to 16 fields of one chunk height (pcr_apply_batched),
    # then the 16 Poisson solves stage by stage, one launch per transform
    # length, z-solve shape and chunk count (poisson_solve_batched)
    from paper_2502_06296_amd import autotune
    log("bench: uneven batch, grouped launches")
    by_m = {}
    for tk in tasks:
        for pl, fl in zip(tk["pcr"], tk["fields"]):
            by_m.setdefault(autotune.pcr_shape(pl)[0], []).append((pl, fl))
    hgroups = []
    for items in by_m.values():
        for k in range(0, len(items), 16):
            hgroups.append(([pl for pl, _ in items[k:k + 16]], [fl for _, fl in items[k:k + 16]]))
    pplans = [tk["poisson"] for tk in tasks]
    prhs = [tk["rhs"] for tk in tasks]
    pout = [tk["p"] for tk in tasks]

    def grouped():
        with torch.cuda.stream(stream):
            for pls, fls in hgroups:
                pf.pcr_apply_batched(pls, fls)
            pf.poisson_solve_batched(pplans, prhs, pout)

    for _ in range(args.warmup):
        grouped()
    stream.synchronize()
    a.record(stream)
    for _ in range(args.steps):
        grouped()
    b.record(stream)
    stream.synchronize()
    ms = a.elapsed_time(b) / args.steps
    pf.pf_graph_begin(stream)
    grouped()
    gr = pf.pf_graph_end(stream)
    gr.launch(stream)
    stream.synchronize()
    a.record(stream)
    for _ in range(args.steps):
        gr.launch(stream)
    b.record(stream)
    stream.synchronize()
    gms = a.elapsed_time(b) / args.steps
    grow = {"helmholtz_launches": len(hgroups), "ms": round(ms, 3), "graph_ms": round(gms, 3),
            "gpoints_per_s": round(pts / ms / 1e6, 2), "graph_gpoints_per_s": round(pts / gms / 1e6, 2)}
    print(json.dumps({"workload": f"16 uneven problems ({pts} points): Poisson + 3 Helmholtz each, FP32+refine",
                      "metric": "Gpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "by_lanes": rows, "grouped_one_stream": grow}), flush=True)


SHARES = {
    # the paper's per-GPU share of its weak-scaling runs (Sec. 3.1)
    "weak_share": ((3456, 3072, 30), "weak-scaling share"),
    # one z slab of its strong-scaling grid 3200 x 3456 x 900 over 32 GPUs
    # (Sec. 3.1, 1-D slabs): 28 planes (four of the 32 slabs hold 29)
    "strong_slab": ((3200, 3456, 28), "strong-scaling slab of 3200x3456x900 over 32 GPUs,"),
}


def per_gpu_share(args):
    """One GPU's share of the paper's scaling runs (Sec. 3.1): the headline
    step (3 Helmholtz + Poisson) in both precisions, and the Helmholtz apply
    with 1, 2 and 4 chunks per column (one chunk is a plain elimination;
    more chunks add the reduced system)."""
    global NX, NY, NZ
    (NX, NY, NZ), label = SHARES[args.workload]
    import torch
    import paper_2502_06296_amd as pf
    from paper_2502_06296_amd import autotune
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    f = device_rhs(torch, dev, (NZ, NY, NX))
    npts = NX * NY * NZ
    out = {"workload": f"{label} {NX}x{NY}x{NZ}, tanh 1.5: 3 z-Helmholtz + pressure Poisson",
           "metric": "Gpoints/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup}
    for prec in ("fp32_refine", "fp64"):
        log(f"{args.workload}: {prec}")
        st = Step(pf, torch, dev, prec, f, tune=not args.no_tune)
        ms, _, stages = time_steps(st, args.steps, args.warmup)
        entry = {"value": round(npts / (ms * 1e-3) / 1e9, 3), "ms_per_step": round(ms, 4),
                 "stages_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in stages.items()},
                 "autotuned": st.tuned}
        chunking = {}
        for rows in (32, 16, 8):
            if not autotune.set_pcr_shape(st.pcr, rows, 64):
                continue
            ms_c, _, stg = time_steps(st, args.steps, 1)
            chunking[f"chunk_rows_{rows}_P{(NZ + rows - 1) // rows}"] = round(stg["pcr_apply"][0] / stg["pcr_apply"][1], 4)
        entry["pcr_apply_ms_by_chunking"] = chunking
        out[prec] = entry
        del st
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def slab_rel_l2(torch, a, b, slab=64):
    """||a - b|| / ||b|| accumulated over z slabs (bounded temporaries)."""
    num = den = 0.0
    for k in range(0, a.shape[0], slab):
        d = a[k:k + slab] - b[k:k + slab]
        num += float(torch.sum(d * d))
        den += float(torch.sum(b[k:k + slab] * b[k:k + slab]))
        del d
    return (num / den) ** 0.5


def helmholtz_c3(torch, pf, dev, steps, warmup):
    """The three-component z-Helmholtz of the 1024 x 1024 x 512 grid (u, v
    centres, w faces) in one batched launch, per precision."""
    nx, ny, nz = HELM_C3
    out = {"workload": f"3 z-Helmholtz (u, v centres; w faces) in one launch, {nx}x{ny}x{nz}, "
                       f"tanh {BETA}, s = {S_HELM:.4g}"}
    pts = nx * ny * (3 * nz - 1)
    for prec in ("fp32_refine", "fp64", "fp32"):
        log(f"bench: helmholtz {nx}x{ny}x{nz} {prec}")
        dt = torch.float32 if prec == "fp32" else torch.float64
        st = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(st):
            plans = []
            for bc in ("dirichlet_centre", "dirichlet_centre", "dirichlet_face"):
                al, ga, ex = pf.zop_rows(nz, bc, LZ, BETA)
                plans.append(pf.pcr_prepare(al, ga, ex, S_HELM, precision=prec, stream=st))
            u = [torch.empty((nz if c < 2 else nz - 1, ny, nx), dtype=dt, device=dev) for c in range(3)]
            for c, x in enumerate(u):
                fill_normal(torch, x, HELM_SEED + c)
            for _ in range(warmup):
                pf.pcr_apply_batched(plans, u)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            for _ in range(steps):
                pf.pcr_apply_batched(plans, u)
            b.record(st)
        b.synchronize()
        ms = a.elapsed_time(b) / steps
        bpp = 8 if prec == "fp32" else 16
        out[prec] = {"ms": round(ms, 4), "gpoints_per_s": round(pts / ms / 1e6, 3),
                     "gbs": round(bpp * pts / ms / 1e6, 1)}
        del plans, u
        torch.cuda.empty_cache()
    return out


TUNE_CACHE = os.path.join(tempfile.gettempdir(), "pf_channel_bench_tune.json")


def headline(args):
    """The projection step at the workload's grid, FP32+refine then FP64 (one
    precision's plans and fields freed before the other's are built)."""
    import torch
    import paper_2502_06296_amd as pf

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"bench: {NX}x{NY}x{NZ}: generating inputs on the device")
    f = device_rhs(torch, dev, (NZ, NY, NX))
    traffic = None
    if os.path.exists(traffic_file()):
        with open(traffic_file()) as fh:
            traffic = json.load(fh)

    results, kept = {}, {}
    for prec in (["fp32_refine"] if args.no_fp64 else ["fp32_refine", "fp64"]):
        log(f"bench: {prec} plans")
        st = Step(pf, torch, dev, prec, f, tune=not args.no_tune)
        if st.tuned:
            log(f"bench: {prec} autotuned shapes {st.tuned}")
        ms, wall, stages = time_steps(st, args.steps, args.warmup)
        log(f"bench: {prec} {ms:.3f} ms/step")
        gms = graph_ms(st, max(3, args.steps // 2))
        # accuracy of the timed configuration: one fresh step
        st.reset_fields()
        st.run()
        st.stream.synchronize()
        kept[prec] = (st.p, st.u)
        results[prec] = dict(ms=ms, wall=wall, stages=stages, graph_ms=gms, tuned=st.tuned)
        del st
        torch.cuda.empty_cache()

    acc = {}
    if "fp64" in kept:
        log("bench: accuracy against the float64 GPU path")
        p32, u32 = kept["fp32_refine"]
        p64, u64 = kept["fp64"]
        acc["poisson_rel_l2_vs_fp64_gpu"] = slab_rel_l2(torch, p32, p64)
        acc["helmholtz_rel_l2_vs_fp64_gpu"] = max(slab_rel_l2(torch, a, b) for a, b in zip(u32, u64))
    kept.clear()
    del f
    torch.cuda.empty_cache()

    main = results["fp32_refine"]
    npts = NX * NY * NZ
    value = npts / (main["ms"] * 1e-3) / 1e9
    line = {
        "metric": "Poisson+Helmholtz Gpoints/s, FP32+refine vs FP64 on 1 GPU at rel.err<=1e-10",
        "value": round(value, 3), "unit": "Gpoints/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(main["ms"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64-residual", "data": "synthetic",
        "config": {"workload": f"projection step: 3 z-Helmholtz (u,v centres; w faces; one batched "
                               f"launch) + pressure Poisson, {NX}x{NY}x{NZ} channel, tanh {BETA}, "
                               "float32 with one float64-residual correction and a float64 zero mode",
                   "nx": NX, "ny": NY, "nz": NZ, "beta": BETA, "s": S_HELM,
                   "precision": "fp32_refine", "parallelism": "1 GPU",
                   "inputs": "seeded device draws: f uniform[-1,1] mean removed, u v w N(0,1)"},
        "roofline": roofline("fp32_refine", main["stages"], traffic),
        "stages_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in main["stages"].items()},
        "graph_ms_per_step": round(main["graph_ms"], 4),
        "autotuned": main["tuned"],
        "accuracy": acc,
    }
    if "fp64" in results:
        r64 = results["fp64"]
        line["fp64"] = {"value": round(npts / (r64["ms"] * 1e-3) / 1e9, 3),
                        "ms_per_step": round(r64["ms"], 4),
                        "graph_ms_per_step": round(r64["graph_ms"], 4),
                        "stages_ms_per_launch": {k: round(v[0] / v[1], 4) for k, v in r64["stages"].items()},
                        "autotuned": r64["tuned"],
                        "roofline": roofline("fp64", r64["stages"], traffic)}
        line["speedup_fp32_refine_vs_fp64"] = round(r64["ms"] / main["ms"], 4)
    return line, torch, pf, dev


def side_entries(args, line, torch, pf, dev):
    """The coupled substep and the 3-D Helmholtz on the step's grid."""
    npts = NX * NY * NZ
    coupled = {}
    for prec in (["fp32_refine"] if args.no_fp64 else ["fp32_refine", "fp64"]):
        log(f"bench: coupled step {prec}")
        cs = CoupledStep(pf, torch, dev, prec)
        ms, _, stages = time_steps(cs, args.steps, args.warmup)
        per = {k: round(v[0] / v[1], 4) for k, v in stages.items()}
        pj = per.get("project")
        coupled[prec] = {"ms_per_step": round(ms, 4),
                         "gpoints_per_s": round(npts / (ms * 1e-3) / 1e9, 3),
                         "stages_ms_per_launch": per,
                         "project_gbs": round(COUPLED_BYTES[prec]["project"] * npts / (pj * 1e-3) / 1e9, 1)
                         if pj else None,
                         "xfwd_div_gbs": round(COUPLED_BYTES[prec]["xfwd"] * npts / (per["xfwd"] * 1e-3) / 1e9, 1)}
        del cs
        torch.cuda.empty_cache()
    # the fully implicit variant's Helmholtz (eq. proj2_ustar) of the three
    # components, one 3-D solve each
    h3 = {}
    r3 = [torch.empty((NZ if c < 2 else NZ - 1, NY, NX), dtype=torch.float64, device=dev) for c in range(3)]
    for c, r in enumerate(r3):
        fill_normal(torch, r, HELM_SEED + c)
    for prec in (["fp32_refine"] if args.no_fp64 else ["fp32_refine", "fp64"]):
        log(f"bench: 3-D Helmholtz {prec}")
        plans = [pf.helmholtz3d_plan(NX, NY, NZ, bc, S_HELM, LX, LY, LZ, BETA, precision=prec)
                 for bc in ("dirichlet_centre", "dirichlet_centre", "dirichlet_face")]
        outs3 = [torch.empty_like(r) for r in r3]

        def run3():
            for pl, r, o in zip(plans, r3, outs3):
                pf.helmholtz3d_solve(pl, r, o)
        for _ in range(args.warmup):
            run3()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(args.steps):
            run3()
        b.record()
        torch.cuda.synchronize()
        ms3 = a.elapsed_time(b) / args.steps
        h3[prec] = {"ms_three_components": round(ms3, 4),
                    "gpoints_per_s": round(stage_points("pcr_apply") / (ms3 * 1e-3) / 1e9, 3)}
        del plans, outs3
        torch.cuda.empty_cache()
    line["helmholtz3d"] = {"workload": f"(I - s L) u = r for u, v (centres) and w (faces), 3-D, "
                                       f"{NX}x{NY}x{NZ}, s = {S_HELM:.4g}", **h3}
    line["coupled_step"] = {"workload": "3 z-Helmholtz of (u, v, w) then poisson_project: divergence "
                                        "right-hand side, Poisson, face-gradient correction, pressure "
                                        f"update (gamma dt = {GDT}, c = {C_IMPL:.4g}), same grid",
                            **coupled}


def main():
    global NX, NY, NZ
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes instead of the autotuner's")
    ap.add_argument("--no-coupled", action="store_true",
                    help="channel workload: skip the coupled substep and the 3-D Helmholtz")
    ap.add_argument("--no-helmholtz", action="store_true",
                    help="projection workload: skip the 1024x1024x512 Helmholtz entry")
    ap.add_argument("--copy-calibration", type=int, default=0)
    ap.add_argument("--workload", choices=["projection", "channel", "weak_share", "strong_slab",
                                           "uneven_batch", "ywalls"],
                    default="projection",
                    help="projection: the 2048x1024x1024 step (the headline) and the 1024x1024x512 "
                         "Helmholtz; channel: the 1024x512x512 step with the coupled substep and the "
                         "3-D Helmholtz; weak_share: the paper's per-GPU weak-scaling share "
                         "3456x3072x30; strong_slab: a 3200x3456x28 z slab of its strong-scaling "
                         "grid; uneven_batch: 16 problems of uneven sizes on 1-8 internal streams, "
                         "eager and from one graph; ywalls: the Poisson solve with periodic y and "
                         "with y walls")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one MI355X; runs on more than one GPU are not "
              "supported (the solver is single-device).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload in SHARES:
        per_gpu_share(args)
        return
    if args.workload == "uneven_batch":
        uneven_batch(args)
        return
    if args.workload == "ywalls":
        NX, NY, NZ = SHAPES["channel"]
        ywalls(args)
        return
    NX, NY, NZ = SHAPES[args.workload]
    # the oracle's baseline runs first, in forked workers, before anything
    # touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: oracle cpu baseline")
        cpu = cpu_baseline(NZ)
    line, torch, pf, dev = headline(args)
    if args.workload == "projection" and not args.no_helmholtz:
        line["helmholtz_1024x1024x512"] = helmholtz_c3(torch, pf, dev, args.steps, args.warmup)
    if args.workload == "channel" and not args.no_coupled:
        side_entries(args, line, torch, pf, dev)
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
