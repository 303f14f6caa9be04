"""Packed real Fourier transform (paper App. A).

A real line of n values has floor(n/2)+1 complex Fourier coefficients X_q
(forward sign e^{-2 pi i q t / n}, unnormalised). X_0 is real, and so is
X_{n/2} for even n, so n reals carry the whole spectrum. The packed layout
keeps the interleaved [X_0^r, X_0^i, X_1^r, X_1^i, ...] order and moves the
one surplus value into the always-zero slot of X_0^i:

  even n: [X_0^r, X_{n/2}^r, X_1^r, X_1^i, ..., X_{n/2-1}^r, X_{n/2-1}^i]
  odd n:  [X_0^r, X_h^i,     X_1^r, X_1^i, ..., X_{h-1}^r, X_{h-1}^i, X_h^r]
          with h = (n-1)/2.

The inverse returns the real line, normalised by 1/n. numpy's FFT serves as
the library transform; ``dft_direct`` is a direct summation used to pin it.
"""
from __future__ import annotations

import numpy as np


def _real_dtype(x):
    return np.longdouble if x.dtype == np.longdouble else np.float64


def rfft_packed(x: np.ndarray, axis: int) -> np.ndarray:
    """Packed forward real transform of ``x`` along ``axis``."""
    x = np.moveaxis(np.asarray(x), axis, -1)
    n = x.shape[-1]
    X = np.fft.rfft(x, axis=-1)
    out = np.empty(x.shape, dtype=_real_dtype(x))
    h = n // 2
    out[..., 0] = X[..., 0].real
    if n % 2 == 0:
        out[..., 1] = X[..., h].real
        out[..., 2::2] = X[..., 1:h].real
        out[..., 3::2] = X[..., 1:h].imag
    else:
        if n > 1:
            out[..., 1] = X[..., h].imag
            out[..., 2::2] = X[..., 1:h + 1].real
            out[..., 3::2] = X[..., 1:h].imag
    return np.moveaxis(out, -1, axis)


def irfft_packed(P: np.ndarray, axis: int) -> np.ndarray:
    """Inverse of ``rfft_packed`` (normalised by 1/n)."""
    P = np.moveaxis(np.asarray(P), axis, -1)
    n = P.shape[-1]
    h = n // 2
    cdt = np.clongdouble if P.dtype == np.longdouble else np.complex128
    X = np.zeros(P.shape[:-1] + (h + 1,), dtype=cdt)
    X[..., 0] = P[..., 0]
    if n % 2 == 0:
        X[..., h] = P[..., 1]
        X[..., 1:h] = P[..., 2::2] + 1j * P[..., 3::2]
    elif n > 1:
        X[..., 1:h] = P[..., 2:-1:2] + 1j * P[..., 3::2]
        X[..., h] = P[..., -1] + 1j * P[..., 1]
    x = np.fft.irfft(X, n=n, axis=-1)
    return np.moveaxis(x, -1, axis)


def dft_direct(x: np.ndarray) -> np.ndarray:
    """Direct O(n^2) summation of the forward DFT of a 1-D sequence."""
    x = np.asarray(x)
    n = x.shape[0]
    t = np.arange(n)
    X = np.zeros(n, dtype=np.complex128)
    for q in range(n):
        X[q] = np.sum(x * np.exp(-2j * np.pi * ((q * t) % n) / n))
    return X


def dct2(x: np.ndarray, axis: int) -> np.ndarray:
    """Cosine transform of ``x`` along ``axis`` for walls at both ends (paper
    Sec. 2.2.1: the cosine member of the Fourier-based transforms), written
    out from its definition: X_q = 2 sum_t x_t cos(pi q (2t + 1) / (2n)),
    q, t = 0..n-1 (the eigenvectors of the second difference with mirrored
    end values). A dense matrix product; ``x`` may be complex."""
    x = np.moveaxis(np.asarray(x), axis, -1)
    n = x.shape[-1]
    t = np.arange(n)
    M = 2.0 * np.cos(np.pi * np.outer(t, 2 * t + 1) / (2 * n))
    return np.moveaxis(x @ M.T, -1, axis)


def idct2(X: np.ndarray, axis: int) -> np.ndarray:
    """Inverse of ``dct2``: x_t = (X_0 / 2 + sum_{q>=1} X_q cos(pi q (2t + 1)
    / (2n))) / n."""
    X = np.moveaxis(np.asarray(X), axis, -1)
    n = X.shape[-1]
    t = np.arange(n)
    M = np.cos(np.pi * np.outer(2 * t + 1, t) / (2 * n))
    M[:, 0] = 0.5
    return np.moveaxis((X @ M.T) / n, -1, axis)


def dst2(x: np.ndarray, axis: int) -> np.ndarray:
    """Sine transform of ``x`` along ``axis`` for walls at both ends where the
    value vanishes (the sine member of Sec. 2.2.1's transforms), from its
    definition: Y_q = 2 sum_t x_t sin(pi (q + 1) (2t + 1) / (2n)), q, t =
    0..n-1 (the eigenvectors of the second difference whose ghost values are
    the negated end values)."""
    x = np.moveaxis(np.asarray(x), axis, -1)
    n = x.shape[-1]
    t = np.arange(n)
    M = 2.0 * np.sin(np.pi * np.outer(t + 1, 2 * t + 1) / (2 * n))
    return np.moveaxis(x @ M.T, -1, axis)


def idst2(Y: np.ndarray, axis: int) -> np.ndarray:
    """Inverse of ``dst2``: x_t = (sum_{q<n-1} Y_q sin(pi (q + 1) (2t + 1) /
    (2n)) + Y_{n-1} (-1)^t / 2) / n."""
    Y = np.moveaxis(np.asarray(Y), axis, -1)
    n = Y.shape[-1]
    t = np.arange(n)
    M = np.sin(np.pi * np.outer(2 * t + 1, t + 1) / (2 * n))
    M[:, n - 1] *= 0.5
    return np.moveaxis((Y @ M.T) / n, -1, axis)


def dst1(x: np.ndarray, axis: int) -> np.ndarray:
    """Type-I sine transform along ``axis`` for a field on the y faces between
    two walls where it vanishes (the face-located velocity of Sec. 2.2.1's
    wall-bounded directions): n rows, row m - 1 holding face m = 1..n-1 (the
    interior faces) and row n - 1 the top wall face. From the definition:
    X_q = 2 sum_{m=1}^{n-1} x_m sin(pi q m / n), q = 1..n-1, written to row
    q - 1; the wall row of x is not read and row n - 1 of X is zero. A dense
    matrix product; ``x`` may be complex."""
    x = np.moveaxis(np.asarray(x), axis, -1)
    n = x.shape[-1]
    m = np.arange(1, n)
    M = np.zeros((n, n))
    M[: n - 1, : n - 1] = 2.0 * np.sin(np.pi * np.outer(m, m) / n)
    return np.moveaxis(x @ M.T, -1, axis)


def idst1(X: np.ndarray, axis: int) -> np.ndarray:
    """Inverse of ``dst1``: x_m = (1 / n) sum_{q=1}^{n-1} X_q sin(pi q m / n)
    on the interior faces; the wall row is zero."""
    X = np.moveaxis(np.asarray(X), axis, -1)
    n = X.shape[-1]
    m = np.arange(1, n)
    M = np.zeros((n, n))
    M[: n - 1, : n - 1] = np.sin(np.pi * np.outer(m, m) / n) / n
    return np.moveaxis(X @ M.T, -1, axis)
