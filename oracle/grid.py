"""Grid metrics and second-order operators (paper Sec. 2.1, eq. fijk_eq).

Staggered (MAC) channel grid: uniform spacing in x and y, faces ``zf[0..nz]``
in z. Pressure and the wall-parallel velocities live at cell centres
(``nz`` unknowns), the wall-normal velocity at the interior faces
(``nz - 1`` unknowns).

Every z operator is returned in sign-normalised form: row k of -L_z is

    -alpha[k] * x[k-1] + (alpha[k] + gamma[k] + excess[k]) * x[k] - gamma[k] * x[k+1]

with alpha, gamma, excess >= 0, alpha[0] = gamma[-1] = 0. ``excess`` holds
the wall terms of Dirichlet rows; it is zero for the Neumann (pressure)
operator, whose rows sum to zero.
"""
from __future__ import annotations

import numpy as np

NEUMANN = 0            # pressure, cell centres, zero normal gradient at walls
DIRICHLET_CENTRE = 1   # u, v at cell centres, value 0 at the walls
DIRICHLET_FACE = 2     # w at interior faces, w = 0 on the wall faces

Y_PERIODIC = 0         # y periodic (the channel)
Y_WALLS = 1            # zero-gradient (Neumann) walls at both y ends, cell centres
Y_DIRICHLET = 2        # value-zero (Dirichlet) walls at both y ends, cell centres
Y_FACES = 3            # value-zero walls at both y ends, unknowns on the y faces
                       # (row j is face j + 1; row ny - 1 is the top wall face)

X_PERIODIC = 0         # x periodic (the channel)
X_WALLS = 1            # zero-gradient walls at both x ends, cell centres
X_DIRICHLET = 2        # value-zero walls at both x ends, cell centres
X_FACES = 3            # value-zero walls at both x ends, unknowns on the x faces
                       # (column i is face i + 1; column nx - 1 is the east wall face)


def z_metrics(zf, dtype=np.float64):
    """Centres zc, cell widths dzf (nz), centre distances dzc (nz-1)."""
    zf = np.asarray(zf, dtype=dtype)
    zc = (zf[1:] + zf[:-1]) / 2
    return zc, np.diff(zf), np.diff(zc)


def zop(zf, bc, dtype=np.float64):
    """(alpha, gamma, excess) of -L_z for boundary family ``bc``."""
    zc, dzf, dzc = z_metrics(zf, dtype)
    nz = dzf.size
    one = dtype(1)
    if bc in (NEUMANN, DIRICHLET_CENTRE):
        alpha = np.zeros(nz, dtype)
        gamma = np.zeros(nz, dtype)
        alpha[1:] = one / (dzf[1:] * dzc)      # flux through the lower face
        gamma[:-1] = one / (dzf[:-1] * dzc)    # flux through the upper face
        excess = np.zeros(nz, dtype)
        if bc == DIRICHLET_CENTRE:
            # ghost value mirrored through the wall: the wall flux uses half a
            # cell, 2 / dzf^2 on the diagonal
            excess[0] = 2 * one / (dzf[0] * dzf[0])
            excess[-1] = 2 * one / (dzf[-1] * dzf[-1])
        return alpha, gamma, excess
    if bc == DIRICHLET_FACE:
        # unknown u = 0..nz-2 sits on face k = u+1; control volume dzc[u]
        n = nz - 1
        alpha = one / (dzc * dzf[:-1])
        gamma = one / (dzc * dzf[1:])
        excess = np.zeros(n, dtype)
        excess[0] = alpha[0]          # neighbour w_0 = 0 drops out
        excess[-1] = gamma[-1]        # neighbour w_nz = 0 drops out
        alpha = alpha.copy()
        gamma = gamma.copy()
        alpha[0] = 0
        gamma[-1] = 0
        return alpha, gamma, excess
    raise ValueError(f"unknown boundary family {bc}")


def packed_modes(n: int) -> np.ndarray:
    """Fourier mode index held by each slot of the packed real layout (App. A).

    Even n: slot 0 -> 0, slot 1 -> n/2, slots 2q, 2q+1 -> q.
    Odd n:  slot 0 -> 0, slot 1 -> (n-1)/2 (its imaginary part),
            slots 2q, 2q+1 -> q, slot n-1 -> (n-1)/2 (its real part).
    """
    s = np.arange(n)
    q = s // 2
    q[0] = 0
    if n > 1:
        q[1] = n // 2
    return q


def modified_wavenumbers(n: int, length, dtype=np.float64) -> np.ndarray:
    """sigma per packed slot: 4 sin^2(pi q / n) / dx^2 (minus the second-order
    eigenvalue of the periodic second difference, Schumann & Sweet)."""
    q = packed_modes(n).astype(dtype)
    dx = dtype(length) / dtype(n)
    pi = np.pi if dtype is np.float64 else dtype("3.14159265358979323846264338327950288")
    s = np.sin(pi * q / dtype(n))
    return 4 * s * s / (dx * dx)


def wall_wavenumbers(n: int, length, dtype=np.float64) -> np.ndarray:
    """sigma per cosine mode q = 0..n-1 (natural order) of the cell-centred
    second difference with zero-gradient walls: 4 sin^2(pi q / (2n)) / dx^2."""
    q = np.arange(n, dtype=dtype)
    dx = dtype(length) / dtype(n)
    s = np.sin(np.pi * q / (2 * dtype(n)))
    return 4 * s * s / (dx * dx)


def face_wall_wavenumbers(n: int, length, dtype=np.float64) -> np.ndarray:
    """sigma per type-I sine mode of the second difference on the n - 1
    interior y faces between two walls where the value vanishes: mode q =
    1..n-1 in row q - 1, 4 sin^2(pi q / (2n)) / dy^2. Row n - 1 (the wall
    face, no mode) gets the value of q = n, 4 / dy^2."""
    q = np.arange(n, dtype=dtype) + 1
    dx = dtype(length) / dtype(n)
    s = np.sin(np.pi * q / (2 * dtype(n)))
    return 4 * s * s / (dx * dx)


def dirichlet_wall_wavenumbers(n: int, length, dtype=np.float64) -> np.ndarray:
    """sigma per sine mode q = 0..n-1 (natural order) of the cell-centred
    second difference whose ghost values negate the end values (value zero on
    the walls): 4 sin^2(pi (q + 1) / (2n)) / dx^2."""
    q = np.arange(n, dtype=dtype) + 1
    dx = dtype(length) / dtype(n)
    s = np.sin(np.pi * q / (2 * dtype(n)))
    return 4 * s * s / (dx * dx)
