"""Tridiagonal solvers along axis 0 (paper Sec. 2.2.4, Algorithms 1 and 2).

Two row conventions appear here:

* plain rows  ``a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k]`` (eq.
  eq_tridiag_base), used by the paper's algorithms exactly as stated;
* sign-normalised M-matrix rows
  ``-alpha[k] x[k-1] + (alpha[k] + gamma[k] + eps[k]) x[k] - gamma[k] x[k+1] = d[k]``
  with alpha, gamma, eps >= 0. Every discrete operator of this solver has
  this form. Eliminating in it never forms a diagonal by subtraction: the
  pivot is carried as gamma[k] + g[k] with g[k] = eps[k] +
  alpha[k] g[k-1] / pivot[k-1] >= 0 (the tridiagonal case of the
  Grassmann-Taksar-Heyman elimination, 1985). A plain Thomas sweep on the
  same rows loses digits to the cancellation B - A C / b when eps is small.

Coefficient arrays are indexed by row along axis 0 and broadcast against
``d``'s trailing axes, so one call solves many columns.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- Thomas
def thomas_gth(alpha, gamma, eps, d):
    """Subtraction-free Thomas solve of sign-normalised rows. The system ends
    at its first and last rows, so alpha[0] and gamma[-1] must be zero."""
    d = np.asarray(d)
    n = d.shape[0]
    if np.any(np.asarray(alpha[0]) != 0) or np.any(np.asarray(gamma[n - 1]) != 0):
        raise ValueError("alpha[0] and gamma[-1] must be zero")
    y = np.empty_like(d)
    ratio = np.empty(np.broadcast_shapes(np.shape(gamma[0]), d.shape[1:], np.shape(eps[0])),
                     dtype=d.dtype)
    ratio = np.broadcast_to(ratio, (n,) + ratio.shape).copy()
    g = eps[0] + 0 * d[0]
    piv = gamma[0] + g
    y[0] = d[0] / piv
    ratio[0] = gamma[0] / piv
    for k in range(1, n):
        g = eps[k] + alpha[k] * g / piv
        piv = gamma[k] + g
        y[k] = (d[k] + alpha[k] * y[k - 1]) / piv
        ratio[k] = gamma[k] / piv
    x = y
    for k in range(n - 2, -1, -1):
        x[k] = y[k] + ratio[k] * x[k + 1]
    return x


def thomas_plain(a, b, c, d):
    """Textbook Thomas sweep for plain rows (a[0], c[-1] ignored)."""
    d = np.array(d, dtype=np.result_type(b, d), copy=True)
    n = d.shape[0]
    cp = np.empty((n,) + np.broadcast_shapes(np.shape(b[0]), d.shape[1:]), dtype=d.dtype)
    piv = b[0] + 0 * d[0]
    cp[0] = (c[0] if n > 1 else 0) / piv
    d[0] = d[0] / piv
    for k in range(1, n):
        piv = b[k] - a[k] * cp[k - 1]
        cp[k] = (c[k] if k < n - 1 else 0) / piv
        d[k] = (d[k] - a[k] * d[k - 1]) / piv
    for k in range(n - 2, -1, -1):
        d[k] = d[k] - cp[k] * d[k + 1]
    return d


def gth_to_plain(alpha, gamma, eps):
    """Plain (a, b, c) rows of the sign-normalised system."""
    return -np.asarray(alpha), np.asarray(alpha) + np.asarray(gamma) + np.asarray(eps), -np.asarray(gamma)


# ------------------------------------------------------------- chunking
def even_bounds(n: int, parts: int):
    """Split rows 0..n-1 into ``parts`` contiguous chunks of near-equal size."""
    edges = [(p * n) // parts for p in range(parts + 1)]
    return [(edges[p], edges[p + 1]) for p in range(parts)]


def _check_bounds(n, bounds):
    assert bounds[0][0] == 0 and bounds[-1][1] == n
    for (s0, e0), (s1, _) in zip(bounds[:-1], bounds[1:]):
        assert e0 == s1
    for s, e in bounds:
        if e - s < 2:
            raise ValueError("every chunk needs at least two rows")


# ----------------------------------------------------------- Algorithm 1
def alg1_solve(a, b, c, d, bounds):
    """Partitioned solve with the paper's original cyclic-reduction step
    (Algorithm 1): each chunk is normalised to unit diagonal and reduced to
    rows that couple only its first and last unknowns; the 2P boundary rows
    form a tridiagonal system solved by Thomas; interiors are rebuilt in
    place. 1-D inputs only (a loop per chunk)."""
    n = len(d)
    _check_bounds(n, bounds)
    a = np.array(a, dtype=float); b = np.array(b, dtype=float)
    c = np.array(c, dtype=float); d = np.array(d, dtype=float)
    for s, e in bounds:
        m = e - s
        A, B, C, D = a[s:e], b[s:e], c[s:e], d[s:e]   # views
        for i in (0, 1):
            A[i] /= B[i]; C[i] /= B[i]; D[i] /= B[i]
        for i in range(2, m):
            r = 1.0 / (B[i] - A[i] * C[i - 1])
            D[i] = r * (D[i] - A[i] * D[i - 1])
            C[i] = r * C[i]
            A[i] = -r * A[i] * A[i - 1]
        for i in range(m - 3, 0, -1):
            D[i] = D[i] - C[i] * D[i + 1]
            A[i] = A[i] - C[i] * A[i + 1]
            C[i] = -C[i] * C[i + 1]
        if m > 2:
            r = 1.0 / (1.0 - A[1] * C[0])
            D[0] = r * (D[0] - C[0] * D[1])
            A[0] = r * A[0]
            C[0] = -r * C[0] * C[1]
        B[:] = 1.0
    # reduced system over X[2p] = first, X[2p+1] = last unknown of chunk p
    ra, rb, rc, rd = [], [], [], []
    for s, e in bounds:
        for row in (s, e - 1):
            ra.append(a[row]); rb.append(1.0); rc.append(c[row]); rd.append(d[row])
    X = thomas_plain(np.array(ra), np.array(rb), np.array(rc), np.array(rd))
    for p, (s, e) in enumerate(bounds):
        x0, xl = X[2 * p], X[2 * p + 1]
        d[s + 1:e - 1] = d[s + 1:e - 1] - a[s + 1:e - 1] * x0 - c[s + 1:e - 1] * xl
        d[s], d[e - 1] = x0, xl
    return d


# ----------------------------------------------------------- Algorithm 2
def alg2_prepare(A, B, C, bounds):
    """Algorithm 2, Step 1 as printed: per chunk, the modified (a, b, c)
    from the original (A, B, C). Returns one dict per chunk. A chunk of two
    rows is already reduced and passes through unchanged."""
    out = []
    for s, e in bounds:
        m = e - s
        Ak, Bk, Ck = (np.array(v[s:e], dtype=float) for v in (A, B, C))
        a, b, c = Ak.copy(), Bk.copy(), Ck.copy()
        if m > 2:
            a[1], b[1] = Ak[1], Bk[1]
            for i in range(2, m):
                b[i] = Bk[i] - Ak[i] * Ck[i - 1] / b[i - 1]
                a[i] = -Ak[i] * a[i - 1] / b[i - 1]
            c[m - 1], c[m - 2] = Ck[m - 1], Ck[m - 2]
            for i in range(m - 3, 0, -1):
                a[i] = a[i] - Ck[i] * a[i + 1] / b[i + 1]
                c[i] = -Ck[i] * c[i + 1] / b[i + 1]
            a[0] = Ak[0]
            b[0] = Bk[0] - Ck[0] * a[1] / Bk[1]
            c[0] = -Ck[0] * c[1] / Bk[1]
        out.append(dict(s=s, e=e, A=Ak, C=Ck, a=a, b=b, c=c))
    return out


def alg2_apply(prep, d):
    """Algorithm 2, Steps 2-4: reduce d in place, solve the boundary system
    by Thomas, rebuild the interior with the stored (a, b, c)."""
    d = np.array(d, dtype=float)
    for ch in prep:
        s, e = ch["s"], ch["e"]
        m = e - s
        D = d[s:e]
        if m > 2:
            for i in range(2, m):
                D[i] = D[i] - ch["A"][i] * D[i - 1] / ch["b"][i - 1]
            for i in range(m - 3, -1, -1):
                D[i] = D[i] - ch["C"][i] * D[i + 1] / ch["b"][i + 1]
    ra, rb, rc, rd = [], [], [], []
    for ch in prep:
        s, e = ch["s"], ch["e"]
        ra += [ch["A"][0], ch["a"][-1]]
        rb += [ch["b"][0], ch["b"][-1]]
        rc += [ch["c"][0], ch["C"][-1]]
        rd += [d[s], d[e - 1]]
    X = thomas_plain(np.array(ra), np.array(rb), np.array(rc), np.array(rd))
    for p, ch in enumerate(prep):
        s, e = ch["s"], ch["e"]
        x0, xl = X[2 * p], X[2 * p + 1]
        sl = slice(1, e - s - 1)
        d[s + 1:e - 1] = (d[s + 1:e - 1] - ch["a"][sl] * x0 - ch["c"][sl] * xl) / ch["b"][sl]
        d[s], d[e - 1] = x0, xl
    return d


# ------------------------------------- Algorithm 2, subtraction-free form
def gth_prepare(alpha, gamma, eps, bounds):
    """Algorithm 2, Step 1, in sign-normalised rows. For each chunk returns
    the interior pivots b (rows 1..m-2), the magnitudes |a| and |c| of the
    couplings to the chunk's first and last unknowns, and the two reduced
    boundary rows as (alpha_R, gamma_R, eps_R) triples. Each diagonal is the
    sum of its non-negative parts: a forward excess e' and a backward excess
    eta are carried through the eliminations instead of being formed by
    subtraction. Coefficients may be 1-D or broadcast over columns."""
    out = []
    for s, e in bounds:
        m = e - s
        al, ga, ep = alpha[s:e], gamma[s:e], eps[s:e]
        if m == 2:
            out.append(dict(s=s, e=e, alpha=al, gamma=ga,
                            row0=(al[0], ga[0], ep[0]), rowl=(al[1], ga[1], ep[1]),
                            b=[], a=[], c=[]))
            continue
        b = [None] * m; a = [None] * m; c = [None] * m
        ef = [None] * m; eta = [None] * m
        a[1] = al[1]; ef[1] = ep[1]; b[1] = ga[1] + al[1] + ep[1]
        for i in range(2, m):
            t = al[i] / b[i - 1]
            a[i] = t * a[i - 1]
            ef[i] = ep[i] + t * ef[i - 1]
            b[i] = ga[i] + a[i] + ef[i]
        c[m - 2] = ga[m - 2]
        eta[m - 2] = ef[m - 2]
        for i in range(m - 3, 0, -1):
            t = ga[i] / b[i + 1]
            a[i] = a[i] + t * a[i + 1]
            c[i] = t * c[i + 1]
            eta[i] = ef[i] + t * eta[i + 1]
        t = ga[0] / b[1]
        c0 = t * c[1]
        eta0 = ep[0] + t * eta[1]
        out.append(dict(s=s, e=e, alpha=al, gamma=ga,
                        row0=(al[0], c0, eta0), rowl=(a[m - 1], ga[m - 1], ef[m - 1]),
                        b=b, a=a, c=c))
    return out


def gth_apply(prep, d):
    """Algorithm 2, Steps 2-4 on sign-normalised rows: forward and backward
    reduction of d, subtraction-free Thomas on the 2P boundary rows, then
    x_i = (d_i + |a_i| x_first + |c_i| x_last) / b_i."""
    d = np.array(d, copy=True)
    for ch in prep:
        s, e = ch["s"], ch["e"]
        m = e - s
        if m == 2:
            continue
        D = d[s:e]
        b, al, ga = ch["b"], ch["alpha"], ch["gamma"]
        for i in range(2, m):
            D[i] = D[i] + al[i] * D[i - 1] / b[i - 1]
        for i in range(m - 3, -1, -1):
            D[i] = D[i] + ga[i] * D[i + 1] / b[i + 1]
    ra, rg, re_, rd = [], [], [], []
    for ch in prep:
        s, e = ch["s"], ch["e"]
        for row, (x_al, x_ga, x_ep) in ((s, ch["row0"]), (e - 1, ch["rowl"])):
            ra.append(x_al + 0 * d[row]); rg.append(x_ga + 0 * d[row])
            re_.append(x_ep + 0 * d[row]); rd.append(d[row])
    X = thomas_gth(np.array(ra), np.array(rg), np.array(re_), np.array(rd))
    for p, ch in enumerate(prep):
        s, e = ch["s"], ch["e"]
        m = e - s
        x0, xl = X[2 * p], X[2 * p + 1]
        for i in range(1, m - 1):
            d[s + i] = (d[s + i] + ch["a"][i] * x0 + ch["c"][i] * xl) / ch["b"][i]
        d[s], d[e - 1] = x0, xl
    return d
