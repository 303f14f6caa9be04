"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no arithmetic of the solver: it draws random numbers and
builds the grid definition a caller would hand to either side.

Counter-based generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014). The value for flat index
``idx`` under ``seed`` is the SplitMix64 finaliser applied to
``seed * 2**40 + idx + 0x9E3779B97F4A7C15`` (mod 2**64); the top 53 bits give
a double in [0, 1). The flat index is x-fastest: ``idx = i + nx*(j + ny*k)``,
i.e. a C-order array of shape (nz, ny, nx).

Grid convention (channel of height ``lz``): face coordinates
``zf[k] = lz/2 * (1 + tanh(beta*(2k/nz - 1)) / tanh(beta))``, k = 0..nz; beta = 0
gives a uniform grid.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state ``x`` (uint64 array), wrapping mod 2**64."""
    z = x + GAMMA
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def unit_uniform(seed: int, start: int, count: int) -> np.ndarray:
    """Doubles in [0,1) for counters start..start+count-1."""
    base = np.uint64((int(seed) << 40) & 0xFFFFFFFFFFFFFFFF)
    idx = np.arange(start, start + count, dtype=np.uint64) + base
    return (splitmix64(idx) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, shape) -> np.ndarray:
    """i.i.d. uniform[-1, 1] array of C-order ``shape`` (flat index = counter)."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float64)
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        out[s:s + c] = 2.0 * unit_uniform(seed, s, c) - 1.0
    return out.reshape(shape)


def normal01(seed: int, shape) -> np.ndarray:
    """N(0,1) by Box-Muller from counters 2*idx (radius) and 2*idx+1 (angle)."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float64)
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        u = unit_uniform(seed, 2 * s, 2 * c).reshape(c, 2)
        r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
        out[s:s + c] = r * np.cos(2.0 * np.pi * u[:, 1])
    return out.reshape(shape)


def tanh_faces(nz: int, lz: float = 2.0, beta: float = 1.5) -> np.ndarray:
    """Face coordinates zf[0..nz] of the wall-clustered channel grid."""
    k = np.arange(nz + 1, dtype=np.float64)
    if beta == 0.0:
        return lz * k / nz
    return 0.5 * lz * (1.0 + np.tanh(beta * (2.0 * k / nz - 1.0)) / np.tanh(beta))


def remove_weighted_mean(f: np.ndarray, zf: np.ndarray) -> np.ndarray:
    """Shift ``f`` (nz, ny, nx) in place so that sum_k dzf[k] * sum_ij f = 0."""
    dzf = np.diff(zf)
    plane = f.reshape(f.shape[0], -1).sum(axis=1)
    c = float(np.dot(dzf, plane) / (dzf.sum() * (f.shape[1] * f.shape[2])))
    f -= c
    return f


def channel_rhs(seed: int, nx: int, ny: int, nz: int, lz: float = 2.0,
                beta: float = 1.5):
    """Poisson right-hand side: uniform[-1,1], weighted mean removed. Returns (f, zf)."""
    zf = tanh_faces(nz, lz, beta)
    f = uniform_pm1(seed, (nz, ny, nx))
    remove_weighted_mean(f, zf)
    return f, zf


def draw_uneven_batch(seed: int, count: int = 16):
    """Problem shapes for a batch of uneven channel grids.

    Edge lengths x, y from {64,128,192,256}, z from {96,192,384}, stretching
    factor from [1, 2], all drawn from the counter stream of ``seed``.
    """
    u = unit_uniform(seed ^ 0x5EED, 0, 4 * count).reshape(count, 4)
    xy = np.array([64, 128, 192, 256])
    zz = np.array([96, 192, 384])
    out = []
    for r in u:
        out.append(dict(nx=int(xy[int(r[0] * 4)]), ny=int(xy[int(r[1] * 4)]),
                        nz=int(zz[int(r[2] * 3)]), beta=float(1.0 + r[3])))
    return out
