"""Tridiagonal solvers along axis 0 (paper Sec. 2.2.4, Algorithms 1 and 2).

Two row conventions appear here:

* plain rows  ``a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k]`` (eq.
  eq_tridiag_base), the rows the paper's algorithms take;
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


# ------------------------------------------------------ partitioned solve
# Sec. 2.2.4 (Algorithms 1 and 2, after Laszlo et al.): the rows are split
# into P contiguous chunks. Inside a chunk [s, e) every interior unknown
# (rows s+1..e-2) is expressed through the chunk's two end unknowns, which
# leaves a tridiagonal system of 2P rows over the end unknowns (eq.
# eq_tridiag_redcyc and the reduced system of the text); its solution gives
# the interiors back. Algebraically this is the Schur complement of the
# interior blocks: with T the interior block, x_I = T^-1 d_I - x_s T^-1 (a_{s+1}
# e_1) - x_{e-1} T^-1 (c_{e-2} e_last), substituted into rows s and e-1.
# Algorithms 1 and 2 compute exactly these quantities; Algorithm 2 splits
# them into a coefficient-only part (Step 1, done once per matrix) and a
# part per right-hand side (Steps 2-4), which is the prepare / apply split
# below. The interior blocks here are solved directly (a dense solve for
# plain rows, the subtraction-free Thomas sweep for sign-normalised rows),
# not by the paper's elimination sequence, so that the reduction is checked
# independently of how the GPU reaches it.
def schur_prepare(a, b, c, bounds):
    """Coefficient-only part of the partitioned solve of plain rows (1-D
    coefficients): per chunk the dense interior block T and the two vectors
    q0 = T^-1 (a_{s+1} e_1), ql = T^-1 (c_{e-2} e_last) that carry the end
    unknowns into the interior; and the reduced rows over the 2P end
    unknowns X[2p] = x_s, X[2p+1] = x_{e-1}."""
    a, b, c = (np.asarray(v, dtype=float) for v in (a, b, c))
    n = len(b)
    _check_bounds(n, bounds)
    P = len(bounds)
    R = np.zeros((2 * P, 2 * P))
    chunks = []
    for p, (s, e) in enumerate(bounds):
        m = e - s
        ch = dict(s=s, e=e)
        if m > 2:
            k = np.arange(s + 1, e - 1)
            T = np.diag(b[k]) + np.diag(a[k[1:]], -1) + np.diag(c[k[:-1]], 1)
            rhs = np.zeros((m - 2, 2))
            rhs[0, 0] = a[s + 1]
            rhs[-1, 1] = c[e - 2]
            q = np.linalg.solve(T, rhs)
            ch.update(T=T, q0=q[:, 0], ql=q[:, 1])
            # row s:  a_s x_{s-1} + (b_s - c_s q0[0]) x_s - c_s ql[0] x_{e-1}
            R[2 * p, 2 * p] = b[s] - c[s] * q[0, 0]
            R[2 * p, 2 * p + 1] = -c[s] * q[0, 1]
            # row e-1: -a_{e-1} q0[-1] x_s + (b_{e-1} - a_{e-1} ql[-1]) x_{e-1} + c_{e-1} x_e
            R[2 * p + 1, 2 * p] = -a[e - 1] * q[-1, 0]
            R[2 * p + 1, 2 * p + 1] = b[e - 1] - a[e - 1] * q[-1, 1]
        else:
            R[2 * p, 2 * p], R[2 * p, 2 * p + 1] = b[s], c[s]
            R[2 * p + 1, 2 * p], R[2 * p + 1, 2 * p + 1] = a[e - 1], b[e - 1]
        if p > 0:
            R[2 * p, 2 * p - 1] = a[s]
        if p < P - 1:
            R[2 * p + 1, 2 * p + 2] = c[e - 1]
        chunks.append(ch)
    return dict(a=a, c=c, chunks=chunks, R=R)


def schur_apply(prep, d):
    """Per right-hand side: y = T^-1 d_I per chunk, the reduced right-hand
    sides d_s - c_s y[0] and d_{e-1} - a_{e-1} y[-1], a dense solve of the
    2P reduced rows, then x_I = y - q0 x_s - ql x_{e-1}."""
    d = np.array(d, dtype=float)
    a, c = prep["a"], prep["c"]
    rd = np.empty(len(prep["R"]))
    ys = []
    for p, ch in enumerate(prep["chunks"]):
        s, e = ch["s"], ch["e"]
        y = np.linalg.solve(ch["T"], d[s + 1:e - 1]) if "T" in ch else None
        ys.append(y)
        rd[2 * p] = d[s] - (c[s] * y[0] if y is not None else 0.0)
        rd[2 * p + 1] = d[e - 1] - (a[e - 1] * y[-1] if y is not None else 0.0)
    X = np.linalg.solve(prep["R"], rd)
    for p, (ch, y) in enumerate(zip(prep["chunks"], ys)):
        s, e = ch["s"], ch["e"]
        if y is not None:
            d[s + 1:e - 1] = y - ch["q0"] * X[2 * p] - ch["ql"] * X[2 * p + 1]
        d[s], d[e - 1] = X[2 * p], X[2 * p + 1]
    return d


def schur_solve(a, b, c, d, bounds):
    """The partitioned solve in one call (Algorithm 1's single pass)."""
    return schur_apply(schur_prepare(a, b, c, bounds), d)


# ------------------------------------- partitioned, subtraction-free form
def _interior_rows(alpha, gamma, eps, s, e):
    """Sign-normalised rows of the interior block of chunk [s, e): the
    couplings to the end unknowns leave the block but stay in its diagonal,
    so they join the excess (first row: alpha_{s+1}; last row: gamma_{e-2})."""
    al = np.array(alpha[s + 1:e - 1], copy=True)
    ga = np.array(gamma[s + 1:e - 1], copy=True)
    ep = np.array(eps[s + 1:e - 1], copy=True)
    ep[0] = ep[0] + al[0]
    al[0] = 0 * al[0]
    ep[-1] = ep[-1] + ga[-1]
    ga[-1] = 0 * ga[-1]
    return al, ga, ep


def gth_prepare(alpha, gamma, eps, bounds):
    """Coefficient-only part of the partitioned solve in sign-normalised rows
    (-alpha x[k-1] + (alpha + gamma + eps) x[k] - gamma x[k+1] = d[k]).

    The interior block T is itself such an M-matrix, so u0 = T^-1 (alpha_{s+1}
    e_1), ul = T^-1 (gamma_{e-2} e_last) and v = T^-1 eps_I are non-negative,
    and T 1 = eps_I + alpha_{s+1} e_1 + gamma_{e-2} e_last gives v + u0 + ul =
    1. The reduced row of x_s then has the diagonal alpha_s + eps_s + gamma_s
    (1 - u0[0]) = alpha_s + gamma_s ul[0] + (eps_s + gamma_s v[0]): its
    off-diagonal parts alpha_s and gamma_s ul[0] and a non-negative excess,
    with no subtraction; the row of x_{e-1} mirrors it. Coefficients may be
    1-D or broadcast over columns (trailing axes)."""
    out = []
    for s, e in bounds:
        if e - s < 2:
            raise ValueError("every chunk needs at least two rows")
        ch = dict(s=s, e=e)
        if e - s == 2:
            ch["row0"] = (alpha[s], gamma[s], eps[s])
            ch["rowl"] = (alpha[e - 1], gamma[e - 1], eps[e - 1])
        else:
            al, ga, ep = _interior_rows(alpha, gamma, eps, s, e)
            mI = e - s - 2
            shape = np.broadcast_shapes(np.shape(alpha[s]), np.shape(gamma[s]), np.shape(eps[s]))
            rhs = np.zeros((mI, 3) + shape)
            rhs[:, 0] = eps[s + 1:e - 1]
            rhs[0, 1] = alpha[s + 1]
            rhs[-1, 2] = gamma[e - 2]
            sl = (slice(None), None)
            V = thomas_gth(al[sl], ga[sl], ep[sl], rhs)
            v, u0, ul = V[:, 0], V[:, 1], V[:, 2]
            ch.update(T=(al, ga, ep), u0=u0, ul=ul, gs=gamma[s], al_l=alpha[e - 1])
            ch["row0"] = (alpha[s], gamma[s] * ul[0], eps[s] + gamma[s] * v[0])
            ch["rowl"] = (alpha[e - 1] * u0[-1], gamma[e - 1], eps[e - 1] + alpha[e - 1] * v[-1])
        out.append(ch)
    return out


def gth_apply(prep, d):
    """Per right-hand side: y = T^-1 d_I per chunk, the reduced right-hand
    sides d_s + gamma_s y[0] and d_{e-1} + alpha_{e-1} y[-1], the
    subtraction-free Thomas sweep over the 2P reduced rows, then x_I = y +
    u0 x_s + ul x_{e-1}."""
    d = np.array(d, copy=True)
    ys = []
    ra, rg, re_, rd = [], [], [], []
    for ch in prep:
        s, e = ch["s"], ch["e"]
        y = None
        d0, dl = d[s], d[e - 1]
        if "T" in ch:
            al, ga, ep = ch["T"]
            y = thomas_gth(al, ga, ep, d[s + 1:e - 1])
            d0 = d0 + ch["gs"] * y[0]
            dl = dl + ch["al_l"] * y[-1]
        ys.append(y)
        for (x_al, x_ga, x_ep), dv in ((ch["row0"], d0), (ch["rowl"], dl)):
            ra.append(x_al + 0 * dv); rg.append(x_ga + 0 * dv)
            re_.append(x_ep + 0 * dv); rd.append(dv)
    X = thomas_gth(np.array(ra), np.array(rg), np.array(re_), np.array(rd))
    for p, (ch, y) in enumerate(zip(prep, ys)):
        s, e = ch["s"], ch["e"]
        if y is not None:
            d[s + 1:e - 1] = y + ch["u0"] * X[2 * p] + ch["ul"] * X[2 * p + 1]
        d[s], d[e - 1] = X[2 * p], X[2 * p + 1]
    return d
