"""Parity bars shared by the GPU tests: every comparison with the oracle checks
the relative L2 error over all points (the bar the results are quoted on)
and, next to it, the largest element-wise error against the largest
reference value, so that an error confined to a few columns or to one slot
pair cannot hide in the global norm.
"""
import numpy as np

TOL = {"fp64": 1e-12, "fp32_refine": 1e-10, "fp32": 1e-5}


def errors(got, ref):
    """(relative L2, max|got - ref| / max|ref|), accumulated in float64."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    nref = np.sqrt(np.sum(ref * ref))
    l2 = np.sqrt(np.sum(d * d)) / nref if nref > 0 else np.sqrt(np.sum(d * d))
    mref = np.max(np.abs(ref)) if ref.size else 0.0
    mx = np.max(np.abs(d)) / mref if mref > 0 else (np.max(np.abs(d)) if d.size else 0.0)
    return float(l2), float(mx)


def check(got, ref, tol, label=""):
    """Assert both bars at tolerance tol; prints the two errors."""
    l2, mx = errors(got, ref)
    print(f"  {label} rel L2 {l2:.3e}, max elementwise {mx:.3e} (tol {tol:.0e})", flush=True)
    assert l2 < tol, (label, l2)
    assert mx < tol, (label, mx)
    return l2, mx
