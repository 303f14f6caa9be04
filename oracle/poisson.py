"""Channel pressure-Poisson and wall-normal Helmholtz solves (paper Sec. 2.2.1,
eq. fijk_eq; Sec. 2.1, eq. proj3_impl1d).

Poisson: find p with L7 p = f, where L7 is the second-order 7-point operator
of the staggered grid -- periodic uniform second differences in x and y plus
the stretched three-point z operator with zero-gradient (Neumann) walls. L7
is singular (constants), so f is first projected onto its range by removing
its dzf-weighted mean, and p is pinned to zero dzf-weighted mean.

Route (method of eigenfunction expansions): packed real transform along x,
then along y (App. A layout); every slot pair (i, j) then decouples into one
tridiagonal system in z whose diagonal is shifted by the modified wavenumbers
sigma_x[i] + sigma_y[j]; the singular (0, 0) system is solved with the pin;
inverse transforms bring p back.

Helmholtz: u - s L_z u = r per column with Dirichlet walls (s = alpha nu dt;
the paper writes gamma_k nu dt / 2).
"""
from __future__ import annotations

import numpy as np

from . import grid, transforms, tridiag


def project_rhs(f, zf):
    """Remove the dzf-weighted mean of f (the part outside L7's range)."""
    _, dzf, _ = grid.z_metrics(zf, f.dtype.type)
    plane = f.reshape(f.shape[0], -1).sum(axis=1)
    c = np.dot(dzf, plane) / (dzf.sum() * (f.shape[1] * f.shape[2]))
    return f - c


def zero_mode_solve(fhat00, zf):
    """Solve L_z m = fhat00 for the singular Neumann column, pinned to
    sum_k dzf[k] m[k] = 0. The right-hand side must be compatible
    (sum_k dzf[k] fhat00[k] = 0). The last equation is dropped and replaced
    by m[nz-1] = 0; a Thomas sweep solves the rest; the weighted mean is
    then subtracted."""
    dt = fhat00.dtype.type
    alpha, gamma, eps = grid.zop(zf, grid.NEUMANN, dt)
    n = fhat00.size
    _, dzf, _ = grid.z_metrics(zf, dt)
    m = np.zeros(n, dtype=dt)
    if n > 1:
        al, ga, ep = alpha[:n - 1].copy(), gamma[:n - 1].copy(), eps[:n - 1].copy()
        ep[-1] = ep[-1] + ga[-1]      # m[n-1] = 0: its coupling stays on the diagonal
        ga[-1] = 0
        m[:n - 1] = tridiag.thomas_gth(al, ga, ep, -fhat00[:n - 1])
    return m - np.dot(dzf, m) / dzf.sum()


def _y_transform(ybc):
    """(forward, inverse, wavenumbers) of the y direction for ybc."""
    if ybc == grid.Y_WALLS:
        return transforms.dct2, transforms.idct2, grid.wall_wavenumbers
    if ybc == grid.Y_DIRICHLET:
        return transforms.dst2, transforms.idst2, grid.dirichlet_wall_wavenumbers
    if ybc == grid.Y_FACES:
        return transforms.dst1, transforms.idst1, grid.face_wall_wavenumbers
    return transforms.rfft_packed, transforms.irfft_packed, grid.modified_wavenumbers


def _x_transform(xbc):
    """(forward, inverse, wavenumbers) of the x direction for xbc: the same
    three members of the Fourier-based transforms as along y."""
    return _y_transform({grid.X_WALLS: grid.Y_WALLS, grid.X_DIRICHLET: grid.Y_DIRICHLET,
                         grid.X_FACES: grid.Y_FACES}.get(xbc, grid.Y_PERIODIC))


def solve_poisson(f, zf, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
    """p with L7 p = f (projected), zero dzf-weighted mean. f is (nz, ny, nx),
    float64 or longdouble; the result has f's dtype. ybc = grid.Y_WALLS puts
    zero-gradient walls at both y ends (cell-centred unknowns): the y
    transform is then the cosine transform and its wavenumbers those of the
    mirrored second difference (Sec. 2.2.1). ybc = grid.Y_DIRICHLET puts walls
    where the value vanishes: the sine transform. xbc does the same for the x
    ends (grid.X_WALLS, grid.X_DIRICHLET). With value-zero walls in x or y, L7
    is nonsingular, so f is not projected and p carries no pin."""
    if ybc == grid.Y_FACES or xbc == grid.X_FACES:
        raise ValueError("the pressure lives at cell centres: faces are for the 3-D Helmholtz")
    dt = f.dtype.type
    nz, ny, nx = f.shape
    singular = ybc != grid.Y_DIRICHLET and xbc != grid.X_DIRICHLET
    if singular:
        f = project_rhs(f, zf)
    xf, xi, xw = _x_transform(xbc)
    yf, yi, yw = _y_transform(ybc)
    F = yf(xf(f, axis=2), axis=1)
    sx = xw(nx, lx, dt)
    sy = yw(ny, ly, dt)
    alpha, gamma, eps = grid.zop(zf, grid.NEUMANN, dt)
    shift = sy[:, None] + sx[None, :]                  # (ny, nx) >= 0
    if singular:
        shift[0, 0] = 1                                # placeholder, redone below
    eps3 = eps[:, None, None] + shift[None, :, :]
    # -(L_z - shift) phi = -fhat in sign-normalised rows
    P = tridiag.thomas_gth(alpha[:, None, None], gamma[:, None, None], eps3, -F)
    if singular:
        P[:, 0, 0] = zero_mode_solve(F[:, 0, 0].copy(), zf)
    return xi(yi(P, axis=1), axis=2)


def apply_L7(p, zf, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
    """L7 p in the arithmetic of p's dtype (x and y each periodic or between
    walls, whose ghost values mirror (zero gradient) or negate (value zero)
    the end values; Neumann z)."""
    dt = p.dtype.type
    nz, ny, nx = p.shape
    dx, dy = dt(lx) / nx, dt(ly) / ny

    def d2(a, axis, bc, walls, value_zero, h):
        if bc in walls:
            sg = -1 if bc == value_zero else 1
            first = np.take(a, [0], axis=axis)
            last = np.take(a, [a.shape[axis] - 1], axis=axis)
            am = np.concatenate([sg * first, np.take(a, range(a.shape[axis] - 1), axis=axis)], axis=axis)
            ap = np.concatenate([np.take(a, range(1, a.shape[axis]), axis=axis), sg * last], axis=axis)
        else:
            am, ap = np.roll(a, 1, axis), np.roll(a, -1, axis)
        return (ap - 2 * a + am) / (h * h)

    out = d2(p, 2, xbc, (grid.X_WALLS, grid.X_DIRICHLET), grid.X_DIRICHLET, dx)
    out += d2(p, 1, ybc, (grid.Y_WALLS, grid.Y_DIRICHLET), grid.Y_DIRICHLET, dy)
    alpha, gamma, eps = grid.zop(zf, grid.NEUMANN, dt)
    lz = -(alpha + gamma + eps)[:, None, None] * p
    lz[1:] += alpha[1:, None, None] * p[:-1]
    lz[:-1] += gamma[:-1, None, None] * p[1:]
    return out + lz


def residual7(p, f, zf, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
    """f - L7 p (f projected first where L7 is singular)."""
    singular = ybc != grid.Y_DIRICHLET and xbc != grid.X_DIRICHLET
    fp = project_rhs(f, zf) if singular else f
    return fp - apply_L7(p, zf, lx, ly, ybc, xbc)


def solve_helmholtz(r, zf, s, bc):
    """u with u - s L_z u = r along z for every column; bc is DIRICHLET_CENTRE
    (nz unknowns) or DIRICHLET_FACE (nz - 1 unknowns)."""
    dt = r.dtype.type
    alpha, gamma, eps = grid.zop(zf, bc, dt)
    s = dt(s)
    shp = (slice(None),) + (None,) * (r.ndim - 1)
    return tridiag.thomas_gth((s * alpha)[shp], (s * gamma)[shp], (1 + s * eps)[shp], r)


def solve_helmholtz3d(r, zf, s, bc, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
    """u with (I - s L) u = r, L the 3-D second-order operator: x and y each
    periodic or with walls (xbc, ybc as for the Poisson solve: a field at
    cell-centre x and y positions), L_z of family bc in z (eq. proj2_ustar,
    the fully implicit diffusion of a Runge-Kutta substep with s = gamma_k nu
    dt / 2). Same route as the Poisson solve: transforms in x and y, then per
    slot pair the z rows (s alpha, s gamma, 1 + s excess + s (sigma_x +
    sigma_y)), all non-negative, so there is no singular column."""
    dt = r.dtype.type
    n, ny, nx = r.shape
    s = dt(s)
    # ybc = grid.Y_FACES (xbc = grid.X_FACES): a field on the y (x) faces, the
    # face-located velocity of a y- (x-) walled grid: the type-I sine
    # transform over the ny - 1 (nx - 1) interior faces; the wall row (column)
    # stays zero
    xf, xi, xw = _x_transform(xbc)
    yf, yi, yw = _y_transform(ybc)
    R = yf(xf(r, axis=2), axis=1)
    sx = xw(nx, lx, dt)
    sy = yw(ny, ly, dt)
    alpha, gamma, eps = grid.zop(zf, bc, dt)
    shift = sy[:, None] + sx[None, :]
    diag = (1 + s * eps)[:, None, None] + s * shift[None, :, :]
    U = tridiag.thomas_gth((s * alpha)[:, None, None], (s * gamma)[:, None, None], diag, R)
    return xi(yi(U, axis=1), axis=2)


def rel_l2(x, ref):
    """||x - ref||_2 / ||ref||_2 over all points, accumulated in float64
    (longdouble if either operand is)."""
    x = np.asarray(x); ref = np.asarray(ref)
    dt = np.longdouble if np.longdouble in (x.dtype.type, ref.dtype.type) else np.float64
    num = np.sqrt(np.sum((x.astype(dt) - ref.astype(dt)) ** 2))
    den = np.sqrt(np.sum(ref.astype(dt) ** 2))
    return float(num / den) if den != 0 else float(num)
