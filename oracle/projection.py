"""Pressure projection of a Runge-Kutta substep on the staggered channel grid
(paper Sec. 2.1: eqs. proj1_Lphi, proj1_ukp1, proj1_Pkp1, and proj2_Pkp1 for
implicit diffusion).

    L7 phi = D u* / gdt,    u = u* - gdt G phi,    p = p_old + phi - c L_z phi

gdt is gamma_k dt. c is 0 for explicit diffusion (proj1_Pkp1); with the
wall-normal diffusion implicit (eq. proj3_impl1d) the pressure update takes
the z part of proj2_Pkp1's correction, c = gamma_k nu dt / 2 with L_z.

Staggering (MAC): u[k, j, i] sits on the x face i+1/2 of cell (i, j, k),
v[k, j, i] on the y face j+1/2, w[m, j, i] on the interior z face m+1
(between cells m and m+1, m = 0..nz-2); w = 0 on the two wall faces. D is
the cell divergence (face fluxes over the cell widths dx, dy, dzf[k]); G is
the face gradient (centre differences over dx, dy and the centre distances
dzc[m]). With these definitions D G is exactly the 7-point operator L7 with
zero-gradient walls.

With ybc = grid.Y_WALLS the y ends are walls too: v[:, ny-1, :] is then the
top wall face, where the flux is zero, so the divergence takes it (and the
bottom wall face below row 0) as zero, the gradient across it is zero and
the projection leaves it unchanged; D G is then L7 with zero-gradient y
walls.

With xbc = grid.X_WALLS the x ends are zero-gradient walls in the same way:
u[:, :, nx-1] is the east wall face, the divergence takes it (and the west
wall face of cell 0) as zero, the gradient across it is zero and the
projection leaves it unchanged; D G is then L7 with zero-gradient x walls.

Plain numpy in the dtype of the inputs; test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import grid, poisson


def divergence(u, v, w, zf, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
    """D (u, v, w) at cell centres, shape (nz, ny, nx)."""
    dt = u.dtype.type
    nz, ny, nx = u.shape
    dx, dy = dt(lx) / nx, dt(ly) / ny
    _, dzf, _ = grid.z_metrics(zf, dt)
    if xbc == grid.X_WALLS:
        ue = u.copy()
        ue[:, :, nx - 1] = 0              # the east wall face
        uw = np.zeros_like(u)
        uw[:, :, 1:] = ue[:, :, :-1]      # the west wall face of cell 0 carries 0
        out = (ue - uw) / dx
    else:
        # west face of cell i is the east face of cell i-1 (periodic)
        out = (u - np.roll(u, 1, axis=2)) / dx
    if ybc == grid.Y_WALLS:
        vn = v.copy()
        vn[:, ny - 1] = 0                 # the top wall face
        vs = np.zeros_like(v)
        vs[:, 1:] = vn[:, :-1]            # the bottom wall face below row 0 carries 0
        out = out + (vn - vs) / dy
    else:
        out = out + (v - np.roll(v, 1, axis=1)) / dy
    top = np.zeros_like(u)
    bot = np.zeros_like(u)
    top[:-1] = w            # face k+1 for cells 0..nz-2; the top wall carries 0
    bot[1:] = w             # face k for cells 1..nz-1; the bottom wall carries 0
    return out + (top - bot) / dzf[:, None, None]


def gradient(phi, zf, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
    """G phi on the faces: (gx, gy) of shape (nz, ny, nx), gz of shape
    (nz - 1, ny, nx) on the interior z faces."""
    dt = phi.dtype.type
    nz, ny, nx = phi.shape
    dx, dy = dt(lx) / nx, dt(ly) / ny
    _, _, dzc = grid.z_metrics(zf, dt)
    gx = (np.roll(phi, -1, axis=2) - phi) / dx
    if xbc == grid.X_WALLS:
        gx[:, :, nx - 1] = 0              # no gradient across the east wall face
    gy = (np.roll(phi, -1, axis=1) - phi) / dy
    if ybc == grid.Y_WALLS:
        gy[:, ny - 1] = 0                 # no gradient across the top wall face
    gz = (phi[1:] - phi[:-1]) / dzc[:, None, None]
    return gx, gy, gz


def lz_neumann(phi, zf):
    """L_z phi with the zero-gradient (pressure) rows."""
    dt = phi.dtype.type
    alpha, gamma, excess = grid.zop(zf, grid.NEUMANN, dt)
    out = -(alpha + gamma + excess)[:, None, None] * phi
    out[1:] += alpha[1:, None, None] * phi[:-1]
    out[:-1] += gamma[:-1, None, None] * phi[1:]
    return out


def project(u, v, w, p, zf, lx, ly, gdt, c=0.0, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
    """One projection: returns (u_new, v_new, w_new, p_new, phi)."""
    dt = u.dtype.type
    f = divergence(u, v, w, zf, lx, ly, ybc, xbc) / dt(gdt)
    phi = poisson.solve_poisson(f, zf, lx, ly, ybc, xbc)
    gx, gy, gz = gradient(phi, zf, lx, ly, ybc, xbc)
    g = dt(gdt)
    return (u - g * gx, v - g * gy, w - g * gz, p + phi - dt(c) * lz_neumann(phi, zf), phi)
