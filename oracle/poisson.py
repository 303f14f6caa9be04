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


def solve_poisson(f, zf, lx, ly, ybc=grid.Y_PERIODIC):
    """p with L7 p = f (projected), zero dzf-weighted mean. f is (nz, ny, nx),
    float64 or longdouble; the result has f's dtype. ybc = grid.Y_WALLS puts
    zero-gradient walls at both y ends (cell-centred unknowns): the y
    transform is then the cosine transform and its wavenumbers those of the
    mirrored second difference (Sec. 2.2.1). ybc = grid.Y_DIRICHLET puts walls
    where the value vanishes: the sine transform; L7 is then nonsingular, so f
    is not projected and p carries no pin."""
    dt = f.dtype.type
    nz, ny, nx = f.shape
    if ybc == grid.Y_DIRICHLET:
        Fx = transforms.rfft_packed(f, axis=2)
        F = transforms.dst2(Fx, axis=1)
        sy = grid.dirichlet_wall_wavenumbers(ny, ly, dt)
        sx = grid.modified_wavenumbers(nx, lx, dt)
        alpha, gamma, eps = grid.zop(zf, grid.NEUMANN, dt)
        eps3 = eps[:, None, None] + (sy[:, None] + sx[None, :])[None, :, :]
        P = tridiag.thomas_gth(alpha[:, None, None], gamma[:, None, None], eps3, -F)
        return transforms.irfft_packed(transforms.idst2(P, axis=1), axis=2)
    f = project_rhs(f, zf)
    Fx = transforms.rfft_packed(f, axis=2)
    if ybc == grid.Y_WALLS:
        F = transforms.dct2(Fx, axis=1)
        sy = grid.wall_wavenumbers(ny, ly, dt)
    else:
        F = transforms.rfft_packed(Fx, axis=1)
        sy = grid.modified_wavenumbers(ny, ly, dt)
    sx = grid.modified_wavenumbers(nx, lx, dt)
    alpha, gamma, eps = grid.zop(zf, grid.NEUMANN, dt)
    shift = sy[:, None] + sx[None, :]                  # (ny, nx) >= 0
    shift[0, 0] = 1                                    # placeholder, redone below
    eps3 = eps[:, None, None] + shift[None, :, :]
    # -(L_z - shift) phi = -fhat in sign-normalised rows
    P = tridiag.thomas_gth(alpha[:, None, None], gamma[:, None, None], eps3, -F)
    P[:, 0, 0] = zero_mode_solve(F[:, 0, 0].copy(), zf)
    Py = transforms.idct2(P, axis=1) if ybc == grid.Y_WALLS else transforms.irfft_packed(P, axis=1)
    return transforms.irfft_packed(Py, axis=2)


def apply_L7(p, zf, lx, ly, ybc=grid.Y_PERIODIC):
    """L7 p in the arithmetic of p's dtype (periodic x; periodic y or, with
    ybc = grid.Y_WALLS, zero-gradient y walls, whose ghost values mirror the
    end rows; Neumann z)."""
    dt = p.dtype.type
    nz, ny, nx = p.shape
    dx, dy = dt(lx) / nx, dt(ly) / ny
    out = (np.roll(p, -1, 2) - 2 * p + np.roll(p, 1, 2)) / (dx * dx)
    if ybc in (grid.Y_WALLS, grid.Y_DIRICHLET):
        # ghost rows beyond the walls: the end rows mirrored (zero gradient)
        # or negated (value zero on the wall)
        sg = -1 if ybc == grid.Y_DIRICHLET else 1
        pm = np.concatenate([sg * p[:, :1], p[:, :-1]], axis=1)     # p[j-1]
        pp = np.concatenate([p[:, 1:], sg * p[:, -1:]], axis=1)     # p[j+1]
        out += (pp - 2 * p + pm) / (dy * dy)
    else:
        out += (np.roll(p, -1, 1) - 2 * p + np.roll(p, 1, 1)) / (dy * dy)
    alpha, gamma, eps = grid.zop(zf, grid.NEUMANN, dt)
    lz = -(alpha + gamma + eps)[:, None, None] * p
    lz[1:] += alpha[1:, None, None] * p[:-1]
    lz[:-1] += gamma[:-1, None, None] * p[1:]
    return out + lz


def residual7(p, f, zf, lx, ly, ybc=grid.Y_PERIODIC):
    """f - L7 p (f projected first where L7 is singular)."""
    fp = f if ybc == grid.Y_DIRICHLET else project_rhs(f, zf)
    return fp - apply_L7(p, zf, lx, ly, ybc)


def solve_helmholtz(r, zf, s, bc):
    """u with u - s L_z u = r along z for every column; bc is DIRICHLET_CENTRE
    (nz unknowns) or DIRICHLET_FACE (nz - 1 unknowns)."""
    dt = r.dtype.type
    alpha, gamma, eps = grid.zop(zf, bc, dt)
    s = dt(s)
    shp = (slice(None),) + (None,) * (r.ndim - 1)
    return tridiag.thomas_gth((s * alpha)[shp], (s * gamma)[shp], (1 + s * eps)[shp], r)


def _y_transform(ybc):
    """(forward, inverse, wavenumbers) of the y direction for ybc."""
    if ybc == grid.Y_WALLS:
        return transforms.dct2, transforms.idct2, grid.wall_wavenumbers
    if ybc == grid.Y_DIRICHLET:
        return transforms.dst2, transforms.idst2, grid.dirichlet_wall_wavenumbers
    return transforms.rfft_packed, transforms.irfft_packed, grid.modified_wavenumbers


def solve_helmholtz3d(r, zf, s, bc, lx, ly, ybc=grid.Y_PERIODIC):
    """u with (I - s L) u = r, L the 3-D second-order operator: periodic in x,
    periodic in y or with y walls (ybc, as for the Poisson solve: a field
    at cell-centre y positions), L_z of family bc in z (eq. proj2_ustar, the
    fully implicit diffusion of a Runge-Kutta substep with s = gamma_k nu dt /
    2). Same route as the Poisson solve: transforms in x and y, then per slot
    pair the z rows (s alpha, s gamma, 1 + s excess + s (sigma_x + sigma_y)),
    all non-negative, so there is no singular column."""
    dt = r.dtype.type
    n, ny, nx = r.shape
    s = dt(s)
    fwd, inv, wavenumbers = _y_transform(ybc)
    R = fwd(transforms.rfft_packed(r, axis=2), axis=1)
    sx = grid.modified_wavenumbers(nx, lx, dt)
    sy = wavenumbers(ny, ly, dt)
    alpha, gamma, eps = grid.zop(zf, bc, dt)
    shift = sy[:, None] + sx[None, :]
    diag = (1 + s * eps)[:, None, None] + s * shift[None, :, :]
    U = tridiag.thomas_gth((s * alpha)[:, None, None], (s * gamma)[:, None, None], diag, R)
    return transforms.irfft_packed(inv(U, axis=1), axis=2)


def rel_l2(x, ref):
    """||x - ref||_2 / ||ref||_2 over all points, accumulated in float64
    (longdouble if either operand is)."""
    x = np.asarray(x); ref = np.asarray(ref)
    dt = np.longdouble if np.longdouble in (x.dtype.type, ref.dtype.type) else np.float64
    num = np.sqrt(np.sum((x.astype(dt) - ref.astype(dt)) ** 2))
    den = np.sqrt(np.sum(ref.astype(dt) ** 2))
    return float(num / den) if den != 0 else float(num)
