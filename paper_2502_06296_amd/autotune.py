"""Autotuner for the launch shapes of the solvers.

It picks, per problem shape and precision, the fastest of the library's
variants for the stages that have more than one:

* the Poisson z solve (rows per thread, columns per workgroup, occupancy
  bound, reciprocal flavour), timed on the plan's own buffers;
* the x and y transforms of the Poisson solve (threads per line, lines per
  workgroup, radix order: four shapes per direction);
* the Helmholtz apply (rows per chunk, columns per chunk).

Winners are kept in a JSON cache keyed by GPU architecture, HIP runtime
version, shape and precision (path: $PF_TUNE_CACHE, else
~/.cache/pf_channel/tune.json). A corrupt or unreadable cache is ignored.
poisson_plan applies a cached entry for its shape and precision by default
(apply_cached_poisson). Tuning runs kernels and may allocate; do it at
set-up, not inside a graph capture.
"""
from __future__ import annotations

import ctypes as C
import json
import os

from . import _native as N
from . import solver

STAGE_XFWD = 0
STAGE_YFWD = 1
STAGE_ZSOLVE = 2


def cache_path():
    return os.environ.get("PF_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pf_channel", "tune.json"))


def _arch_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}|hip{torch.version.hip}"


def load_cache(path=None):
    path = path or cache_path()
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_stage(run, read, stage, reps):
    run()
    read()
    t = {}
    for _ in range(reps):
        run()
    t = read()
    ms, n = t[stage]
    return ms / n


def zsolve_variants(plan):
    cnt = C.c_int32()
    N.check(N.lib().poisson_variant_count(plan.handle, STAGE_ZSOLVE, C.byref(cnt)))
    return list(range(cnt.value))


def set_zsolve_variant(plan, v):
    code = N.lib().poisson_set_variant(plan.handle, STAGE_ZSOLVE, int(v))
    return code == N.PF_OK


def get_zsolve_variant(plan):
    v = C.c_int32()
    N.check(N.lib().poisson_get_variant(plan.handle, STAGE_ZSOLVE, C.byref(v)))
    return v.value


def set_variant(plan, stage, v):
    return N.lib().poisson_set_variant(plan.handle, int(stage), int(v)) == N.PF_OK


def get_variant(plan, stage):
    v = C.c_int32()
    N.check(N.lib().poisson_get_variant(plan.handle, int(stage), C.byref(v)))
    return v.value


def transform_shape_count(plan):
    """Number of transform launch shapes (some fit only some plans)."""
    cnt = C.c_int32()
    N.check(N.lib().poisson_variant_count(plan.handle, STAGE_XFWD, C.byref(cnt)))
    return cnt.value


def tune_transforms(plan, rhs, p, reps=3):
    """Time every transform shape that fits the plan, x and y direction
    separately (the x shape by the x forward, x inverse and residual stages,
    the y shape by both y stages); keep the fastest of each. Returns
    {"x": {shape: ms}, "y": {shape: ms}}."""
    cnt = C.c_int32()
    N.check(N.lib().poisson_variant_count(plan.handle, STAGE_XFWD, C.byref(cnt)))
    stages = {"x": (STAGE_XFWD, ("xfwd", "xinv", "xinv_final", "xfwd_resid")),
              "y": (STAGE_YFWD, ("yfwd", "yinv"))}
    out = {}
    solver.poisson_timing(plan, True)
    try:
        for d, (stage, names) in stages.items():
            times = {}
            for v in range(cnt.value):
                if not set_variant(plan, stage, v):
                    continue
                solver.poisson_solve(plan, rhs, p)
                solver.poisson_timing_read(plan)
                for _ in range(reps):
                    solver.poisson_solve(plan, rhs, p)
                t = solver.poisson_timing_read(plan)
                times[v] = sum(t[n][0] for n in names if n in t) / reps
            best = min(times, key=times.get)
            set_variant(plan, stage, best)
            out[d] = times
    finally:
        solver.poisson_timing(plan, False)
    return out


def tune_poisson(plan, rhs, p, reps=3):
    """Time every z-solve variant that fits the plan on (rhs, p); keep the
    fastest. Returns {variant: ms per launch}."""
    solver.poisson_timing(plan, True)
    times = {}
    try:
        for v in zsolve_variants(plan):
            if not set_zsolve_variant(plan, v):
                continue
            times[v] = _time_stage(lambda: solver.poisson_solve(plan, rhs, p),
                                   lambda: solver.poisson_timing_read(plan), "zsolve", reps)
    finally:
        solver.poisson_timing(plan, False)
    best = min(times, key=times.get)
    set_zsolve_variant(plan, best)
    return times


def pcr_shape(plan):
    m, cw = C.c_int32(), C.c_int32()
    N.check(N.lib().pcr_get_shape(plan.handle, C.byref(m), C.byref(cw)))
    return m.value, cw.value


def set_pcr_shape(plans, m, cw):
    for pl in plans:
        if N.lib().pcr_set_shape(pl.handle, int(m), int(cw)) != N.PF_OK:
            return False
    return True


def tune_pcr(plans, fields, reps=3):
    """Time each (rows per chunk, columns per chunk) on a batched apply of
    `fields` (which it overwrites); keep the fastest for all plans."""
    import torch
    keep = [f.clone() for f in fields]
    times = {}
    solver.pcr_timing(plans[0], True)
    try:
        for m in (8, 16, 32):
            for cw in (16, 32, 64):
                if not set_pcr_shape(plans, m, cw):
                    continue
                times[(m, cw)] = _time_stage(lambda: solver.pcr_apply_batched(plans, fields),
                                             lambda: solver.pcr_timing_read(plans[0]),
                                             "pcr_apply", reps)
    finally:
        solver.pcr_timing(plans[0], False)
        for f, k in zip(fields, keep):
            f.copy_(k)
        torch.cuda.synchronize()
    best = min(times, key=times.get)
    set_pcr_shape(plans, *best)
    return times


def poisson_key(nx, ny, nz, precision):
    return f"{_arch_key()}|poisson|{nx}x{ny}x{nz}|{precision}"


def pcr_key(n, nx, ny, precision, count):
    return f"{_arch_key()}|pcr|{count}x{n}x{ny}x{nx}|{precision}"


def apply_cached_poisson(plan, nx, ny, nz, precision, path=None):
    """Apply the cached variants (z solve, x and y transform shapes) for this
    shape and precision if the cache holds an entry that fits the plan.
    Returns the applied entry or None."""
    try:
        ent = load_cache(path).get(poisson_key(nx, ny, nz, precision))
    except Exception:  # no device properties (or no torch): nothing to apply
        return None
    if not isinstance(ent, dict):
        return None
    done = {}
    for name, stage in (("zsolve_variant", STAGE_ZSOLVE), ("xshape", STAGE_XFWD), ("yshape", STAGE_YFWD)):
        v = ent.get(name)
        if isinstance(v, int) and set_variant(plan, stage, v):
            done[name] = v
    return done or None


def apply_or_tune_poisson(plan, rhs, p, precision, reps=3, path=None):
    """Use the cached variants for this shape, or tune the z solve and the
    transform shapes and cache them."""
    nz, ny, nx = plan.shape
    key = poisson_key(nx, ny, nz, precision)
    cache = load_cache(path)
    ent = cache.get(key) if isinstance(cache.get(key), dict) else {}
    if "zsolve_variant" in ent and "xshape" in ent and "yshape" in ent:
        done = apply_cached_poisson(plan, nx, ny, nz, precision, path)
        if done and len(done) == 3:
            return {**done, "cached": True}
    times = tune_poisson(plan, rhs, p, reps)
    tt = tune_transforms(plan, rhs, p, reps)
    best = {"zsolve_variant": get_zsolve_variant(plan), "xshape": get_variant(plan, STAGE_XFWD),
            "yshape": get_variant(plan, STAGE_YFWD)}
    cache[key] = {**best, "ms": {str(k): v for k, v in times.items()},
                  "x_ms": {str(k): v for k, v in tt["x"].items()},
                  "y_ms": {str(k): v for k, v in tt["y"].items()}}
    try:
        save_cache(cache, path)
    except OSError:
        pass
    return {**best, "cached": False, "ms": times, "transform_ms": tt}


def apply_or_tune_pcr(plans, fields, precision, reps=3, path=None):
    key = pcr_key(plans[0].n, fields[0].shape[2], fields[0].shape[1], precision, len(plans))
    cache = load_cache(path)
    ent = cache.get(key)
    if isinstance(ent, dict) and "shape" in ent and set_pcr_shape(plans, *ent["shape"]):
        return {"shape": tuple(ent["shape"]), "cached": True}
    times = tune_pcr(plans, fields, reps)
    best = pcr_shape(plans[0])
    cache[key] = {"shape": list(best), "ms": {f"{m}x{cw}": v for (m, cw), v in times.items()}}
    try:
        save_cache(cache, path)
    except OSError:
        pass
    return {"shape": best, "cached": False, "ms": times}
