"""Brute-force assembled operators for tiny grids.

The z operator is written here from its finite-volume definition -- the
difference of the two face fluxes of a control volume divided by its width
-- and not from ``grid.zop``, so that it checks that module rather than
repeating it. Solutions come from numpy.linalg on the dense matrix.
"""
from __future__ import annotations

import numpy as np

NEUMANN, DIRICHLET_CENTRE, DIRICHLET_FACE = 0, 1, 2


def lz_dense(zf, bc):
    """Dense matrix of the z second-derivative operator L_z."""
    zf = np.asarray(zf, dtype=float)
    nz = zf.size - 1
    zc = 0.5 * (zf[1:] + zf[:-1])
    if bc in (NEUMANN, DIRICHLET_CENTRE):
        M = np.zeros((nz, nz))
        for k in range(nz):
            width = zf[k + 1] - zf[k]
            # upper face flux (u[k+1]-u[k]) / (zc[k+1]-zc[k]); at the top wall:
            # zero (Neumann) or (0 - u[k]) / (zf[nz] - zc[k]) (Dirichlet)
            if k + 1 < nz:
                h = zc[k + 1] - zc[k]
                M[k, k + 1] += 1 / (h * width); M[k, k] -= 1 / (h * width)
            elif bc == DIRICHLET_CENTRE:
                M[k, k] -= 1 / ((zf[nz] - zc[k]) * width)
            if k > 0:
                h = zc[k] - zc[k - 1]
                M[k, k - 1] += 1 / (h * width); M[k, k] -= 1 / (h * width)
            elif bc == DIRICHLET_CENTRE:
                M[k, k] -= 1 / ((zc[k] - zf[0]) * width)
        return M
    if bc == DIRICHLET_FACE:
        n = nz - 1
        M = np.zeros((n, n))
        for u in range(n):
            k = u + 1                           # face index
            width = zc[k] - zc[k - 1]
            up = 1 / ((zf[k + 1] - zf[k]) * width)
            dn = 1 / ((zf[k] - zf[k - 1]) * width)
            M[u, u] -= up + dn
            if u + 1 < n:
                M[u, u + 1] += up
            if u > 0:
                M[u, u - 1] += dn
        return M
    raise ValueError(bc)


def periodic_d2(n, h):
    """Dense periodic second difference on n points of spacing h."""
    M = -2 * np.eye(n)
    for i in range(n):
        M[i, (i + 1) % n] += 1
        M[i, (i - 1) % n] += 1
    return M / (h * h)


def wall_d2(n, h, value_zero=False):
    """Dense second difference on n cell centres of spacing h between two
    walls. Zero-gradient walls: no flux through a wall face, so the end rows
    keep one neighbour. value_zero: the value vanishes on the wall face, half
    a cell from the end centre, so the wall flux is (0 - x_end) / (h / 2)."""
    M = np.zeros((n, n))
    for i in range(n):
        if i > 0:
            M[i, i - 1] += 1
            M[i, i] -= 1
        elif value_zero:
            M[i, i] -= 2
        if i < n - 1:
            M[i, i + 1] += 1
            M[i, i] -= 1
        elif value_zero:
            M[i, i] -= 2
    return M / (h * h)


def face_d2(n, h):
    """Dense second difference on the n - 1 interior faces of n cells of
    spacing h between two walls where the value vanishes: each face couples
    to its two neighbours, a wall face counting as zero."""
    m = n - 1
    M = np.zeros((m, m))
    for i in range(m):
        M[i, i] = -2
        if i > 0:
            M[i, i - 1] = 1
        if i < m - 1:
            M[i, i + 1] = 1
    return M / (h * h)


def _d2(n, length, bc):
    """Second difference of one wall-parallel direction: periodic (bc 0),
    between zero-gradient (1) or value-zero (2) walls."""
    return wall_d2(n, length / n, bc == 2) if bc in (1, 2) else periodic_d2(n, length / n)


def l7_dense(nx, ny, zf, lx, ly, ybc=0, xbc=0):
    """Dense 7-point operator for C-order (nz, ny, nx) flattening; ybc and
    xbc: periodic (0), zero-gradient walls (1) or value-zero walls (2) at
    both ends of y and of x."""
    nz = len(zf) - 1
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    Dx = _d2(nx, lx, xbc)
    Dy = _d2(ny, ly, ybc)
    Dz = lz_dense(zf, NEUMANN)
    return (np.kron(Iz, np.kron(Iy, Dx)) + np.kron(Iz, np.kron(Dy, Ix))
            + np.kron(Dz, np.kron(Iy, Ix)))


def poisson_dense(f, zf, lx, ly, ybc=0, xbc=0):
    """Least-squares solution of L7 p = f with the row sum_ijk dzf[k] p = 0
    appended (the solution of the projected problem when f is compatible)."""
    nz, ny, nx = f.shape
    L = l7_dense(nx, ny, zf, lx, ly, ybc, xbc)
    if ybc == 2 or xbc == 2:         # value-zero walls: nonsingular
        return np.linalg.solve(L, f.reshape(-1)).reshape(f.shape)
    w = np.repeat(np.diff(np.asarray(zf, float)), nx * ny)
    # project f onto the range of L (orthogonal to the weights' null vector)
    fv = f.reshape(-1)
    fv = fv - np.dot(w, fv) / w.sum()
    A = np.vstack([L, w[None, :]])
    b = np.concatenate([fv, [0.0]])
    p, *_ = np.linalg.lstsq(A, b, rcond=None)
    return p.reshape(f.shape)


def helmholtz_dense(r, zf, s, bc):
    """Column-wise dense solve of (I - s L_z) u = r along axis 0."""
    M = np.eye(lz_dense(zf, bc).shape[0]) - s * lz_dense(zf, bc)
    shp = r.shape
    return np.linalg.solve(M, r.reshape(shp[0], -1)).reshape(shp)


def helmholtz3d_dense(r, zf, s, bc, lx, ly, ybc=0, xbc=0):
    """Dense solve of (I - s L) u = r, L the 3-D operator of the staggered
    grid: second differences in x and y, each periodic (0) or between
    zero-gradient (1) or value-zero (2) walls, plus L_z of family bc (C-order
    (n, ny, nx) flattening, n = nz or nz - 1). ybc = 3: a field on the y faces
    between value-zero walls (row j the face j + 1, row ny - 1 the top wall
    face, zero in the result); xbc = 3 the same along x."""
    n, ny, nx = r.shape
    # a field on the y (x) faces: unknowns on the interior faces, the wall
    # row (column) is zero
    my = ny - 1 if ybc == 3 else ny
    mx = nx - 1 if xbc == 3 else nx
    Dy = face_d2(ny, ly / ny) if ybc == 3 else _d2(ny, ly, ybc)
    Dx = face_d2(nx, lx / nx) if xbc == 3 else _d2(nx, lx, xbc)
    u = np.zeros(r.shape, dtype=np.result_type(r, np.float64))
    u[:, :my, :mx] = _helm_dense(r[:, :my, :mx], zf, s, bc, Dx, Dy)
    return u


def _helm_dense(r, zf, s, bc, Dx, Dy):
    n, my, mx = r.shape
    Ix, Iy = np.eye(mx), np.eye(my)
    Dz = lz_dense(zf, bc)
    Iz = np.eye(Dz.shape[0])
    L = (np.kron(Iz, np.kron(Iy, Dx)) + np.kron(Iz, np.kron(Dy, Ix))
         + np.kron(Dz, np.kron(Iy, Ix)))
    M = np.eye(L.shape[0]) - s * L
    return np.linalg.solve(M, r.reshape(-1)).reshape(r.shape)
