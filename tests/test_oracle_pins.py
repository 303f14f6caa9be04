"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each check is chosen so that a plausible slip in the oracle -- a dropped
term, a wrong sign or index, a transposed operand, a mis-placed packed slot
-- fails at least one of them (see also test_oracle_mutations.py).
"""
import numpy as np
import pytest

import synth
from oracle import dense, grid, poisson, transforms, tridiag

LX, LY = 2 * np.pi, np.pi


# ------------------------------------------------------------ transforms
def _packed_from_direct(x):
    """Packed layout of App. A built from a direct-summation DFT."""
    n = len(x)
    X = transforms.dft_direct(x)
    out = np.zeros(n)
    out[0] = X[0].real
    h = n // 2
    if n % 2 == 0:
        if n > 1:
            out[1] = X[h].real
        for q in range(1, h):
            out[2 * q], out[2 * q + 1] = X[q].real, X[q].imag
    else:
        if n > 1:
            out[1] = X[h].imag
        for q in range(1, h):
            out[2 * q], out[2 * q + 1] = X[q].real, X[q].imag
        if n > 1:
            out[n - 1] = X[h].real
    return out


@pytest.mark.parametrize("n", list(range(1, 13)) + [16, 18, 24, 27])
def test_packed_fft_matches_direct_dft(n):
    x = synth.uniform_pm1(n, (n,))
    got = transforms.rfft_packed(x, axis=0)
    np.testing.assert_allclose(got, _packed_from_direct(x), rtol=0, atol=1e-12 * n)
    back = transforms.irfft_packed(got, axis=0)
    np.testing.assert_allclose(back, x, rtol=0, atol=1e-14 * n)


@pytest.mark.parametrize("n", [512, 1024, 2048, 3072, 3200, 3456])
def test_packed_fft_matches_direct_dft_at_workload_lengths(n):
    """The lengths the GPU parity tests and the benchmarks run (512-2048,
    3072 and 3456 = 2^7 3^3, 3200 = 2^7 5^2), pinned by direct summation."""
    x = synth.uniform_pm1(7000 + n, (n,))
    got = transforms.rfft_packed(x, axis=0)
    np.testing.assert_allclose(got, _packed_from_direct(x), rtol=0, atol=1e-14 * np.sqrt(n) * 10)
    back = transforms.irfft_packed(got, axis=0)
    np.testing.assert_allclose(back, x, rtol=0, atol=1e-14 * 10)


@pytest.mark.parametrize("n", [8, 9, 64, 96])
def test_packed_parseval(n):
    x = synth.uniform_pm1(3, (n,))
    P = transforms.rfft_packed(x, axis=0)
    w = np.full(n, 2.0)           # interior modes appear twice in the full spectrum
    w[0] = 1.0
    if n % 2 == 0:
        w[1] = 1.0                # X_{n/2} appears once
    assert np.isclose(np.sum(w * P * P) / n, np.sum(x * x), rtol=1e-13)


@pytest.mark.parametrize("n", [6, 7, 16, 12])
def test_modified_wavenumbers_are_eigenvalues_of_periodic_d2(n):
    """Every packed slot's basis line is an eigenvector of the periodic
    second difference with eigenvalue -sigma[slot] (Sec. 2.2.1)."""
    L = 3.7
    sigma = grid.modified_wavenumbers(n, L)
    D = dense.periodic_d2(n, L / n)
    for s in range(n):
        e = np.zeros(n); e[s] = 1.0
        v = transforms.irfft_packed(e, axis=0)
        np.testing.assert_allclose(D @ v, -sigma[s] * v, atol=1e-10 * (1 + sigma[s]))


# ----------------------------------------------------- whole Poisson solve
@pytest.mark.parametrize("shape,beta,seed", [
    ((6, 4, 5), 1.5, 0), ((8, 6, 7), 2.0, 1), ((5, 3, 4), 1.0, 2),
    ((4, 4, 2), 1.5, 3), ((7, 9, 6), 0.0, 4), ((12, 6, 9), 1.2, 5), ((3, 5, 3), 1.7, 6)])
def test_poisson_matches_dense_bruteforce(shape, beta, seed):
    nx, ny, nz = shape
    f, zf = synth.channel_rhs(seed, nx, ny, nz, beta=beta)
    f += 0.3          # an incompatible constant: both sides must project it away
    p = poisson.solve_poisson(f, zf, LX, LY)
    ref = dense.poisson_dense(f, zf, LX, LY)
    assert poisson.rel_l2(p, ref) < 1e-12


def test_poisson_closed_form_eigenfunctions():
    """Uniform z: cos/sin products are exact discrete eigenfunctions."""
    nx, ny, nz = 16, 12, 10
    zf = synth.tanh_faces(nz, 2.0, 0.0)
    dx, dy, dz = LX / nx, LY / ny, 2.0 / nz
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    for q, r, m, ph in [(1, 0, 0, 0.3), (0, 2, 3, 0.0), (3, 5, 1, 1.1), (8, 6, 9, 0.2), (0, 0, 4, 0.0)]:
        f = (np.cos(2 * np.pi * q * i / nx + ph) * np.cos(2 * np.pi * r * j / ny + 0.5 * ph)
             * np.cos(np.pi * m * (k + 0.5) / nz))
        mu = (-4 * np.sin(np.pi * q / nx) ** 2 / dx ** 2 - 4 * np.sin(np.pi * r / ny) ** 2 / dy ** 2
              - 4 * np.sin(np.pi * m / (2 * nz)) ** 2 / dz ** 2)
        p = poisson.solve_poisson(f, zf, LX, LY)
        assert poisson.rel_l2(p, f / mu) < 1e-13, (q, r, m)


def _l7_sparse(nx, ny, zf):
    import scipy.sparse as sp
    nz = len(zf) - 1
    Dz = sp.csr_matrix(dense.lz_dense(zf, dense.NEUMANN))
    Dx = sp.csr_matrix(dense.periodic_d2(nx, LX / nx))
    Dy = sp.csr_matrix(dense.periodic_d2(ny, LY / ny))
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    return (sp.kron(Iz, sp.kron(Iy, Dx)) + sp.kron(Iz, sp.kron(Dy, Ix))
            + sp.kron(Dz, sp.kron(Iy, Ix))).tocsr()


@pytest.mark.parametrize("shape,beta", [((32, 16, 256), 1.5), ((24, 12, 96), 2.0)])
def test_poisson_residual_at_roundoff(shape, beta):
    nx, ny, nz = shape
    f, zf = synth.channel_rhs(7, nx, ny, nz, beta=beta)
    p = poisson.solve_poisson(f, zf, LX, LY)
    r = f.reshape(-1) - _l7_sparse(nx, ny, zf) @ p.reshape(-1)
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-12
    w = np.diff(zf)
    assert abs(np.sum(p * w[:, None, None])) < 1e-12 * np.sum(np.abs(p) * w[:, None, None])


@pytest.mark.parametrize("shape", [(32, 16, 512), (64, 64, 64)])
def test_poisson_long_double_floor(shape):
    nx, ny, nz = shape
    f, zf = synth.channel_rhs(11, nx, ny, nz, beta=1.5)
    p = poisson.solve_poisson(f, zf, LX, LY)
    pl = poisson.solve_poisson(f.astype(np.longdouble), zf.astype(np.longdouble), LX, LY)
    assert poisson.rel_l2(p, pl) < 1e-13


def test_poisson_invariants():
    nx, ny, nz = 12, 8, 16
    f, zf = synth.channel_rhs(21, nx, ny, nz, beta=1.5)
    g, _ = synth.channel_rhs(22, nx, ny, nz, beta=1.5)
    p_f = poisson.solve_poisson(f, zf, LX, LY)
    p_g = poisson.solve_poisson(g, zf, LX, LY)
    # linearity
    p_fg = poisson.solve_poisson(2.0 * f - 3.0 * g, zf, LX, LY)
    assert poisson.rel_l2(p_fg, 2.0 * p_f - 3.0 * p_g) < 1e-13
    # translation invariance in the periodic directions
    p_s = poisson.solve_poisson(np.roll(np.roll(f, 3, axis=2), -2, axis=1), zf, LX, LY)
    assert poisson.rel_l2(p_s, np.roll(np.roll(p_f, 3, axis=2), -2, axis=1)) < 1e-13
    # mirror symmetry of the channel: flipping z of f on a symmetric grid flips p
    p_m = poisson.solve_poisson(f[::-1].copy(), zf, LX, LY)
    assert poisson.rel_l2(p_m, p_f[::-1]) < 1e-12


# --------------------------------------------------------- z solvers
def _random_mmatrix(rng, n, excess_scale):
    al, ga, ep = rng.random(n), rng.random(n), rng.random(n) * excess_scale
    al[0] = 0.0
    ga[-1] = 0.0
    return al, ga, ep


@pytest.mark.parametrize("n", [2, 3, 5, 10, 17, 64, 96])
@pytest.mark.parametrize("excess", [1.0, 1e-3, 1e-8])
def test_tridiagonal_algorithms_equal_dense(n, excess):
    rng = np.random.default_rng(n)
    al, ga, ep = _random_mmatrix(rng, n, excess)
    d = rng.standard_normal(n)
    a, b, c = tridiag.gth_to_plain(al, ga, ep)
    M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    xd = np.linalg.solve(M, d)
    tol = 1e-11 * np.linalg.cond(M) * 1e-4 + 1e-12
    scale = np.abs(xd).max()
    assert np.abs(tridiag.thomas_gth(al, ga, ep, d) - xd).max() < tol * scale
    chunkings = [tridiag.even_bounds(n, P) for P in (1, 2, 3, 4, 5, 8) if n // P >= 2]
    if n >= 7:
        chunkings.append([(0, 2), (2, 5), (5, n)])          # uneven, with a 2-row chunk
    for bnd in chunkings:
        x1 = tridiag.schur_solve(a, b, c, d, bnd)
        x2 = tridiag.gth_apply(tridiag.gth_prepare(al, ga, ep, bnd), d)
        for x in (x1, x2):
            assert np.abs(x - xd).max() < 1e3 * tol * scale


def test_subtraction_free_pivots_keep_digits():
    """On the stretched pressure operator with a small wavenumber shift the
    plain pivot B - A C / b cancels; the subtraction-free recursion does
    not (the reading that every diagonal is carried as a sum)."""
    nz = 1024
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    al, ga, ep = grid.zop(zf, grid.NEUMANN)
    ep = ep + 4 * np.sin(np.pi / 256) ** 2 / (LX / 256) ** 2
    d = synth.uniform_pm1(5, (nz,))
    ld = np.longdouble
    ref = tridiag.thomas_gth(al.astype(ld), ga.astype(ld), ep.astype(ld), d.astype(ld))
    gth = tridiag.thomas_gth(al, ga, ep, d)
    a, b, c = tridiag.gth_to_plain(al, ga, ep)
    plain = tridiag.thomas_plain(a, b, c, d)
    e_gth = poisson.rel_l2(gth, ref)
    e_plain = poisson.rel_l2(plain, ref)
    assert e_gth < 1e-14
    assert e_plain > 10 * e_gth


@pytest.mark.parametrize("P", [1, 4, 8, 32])
def test_partitioned_subtraction_free_keeps_digits(P):
    """The partitioned solve in sign-normalised rows (every reduced diagonal a
    sum of non-negative parts) keeps the digits of the long-double solve on
    the stretched pressure operator with a small wavenumber shift, where the
    plain Schur complement (diagonals b - c q) loses them."""
    nz = 1024
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    al, ga, ep = grid.zop(zf, grid.NEUMANN)
    ep = ep + 4 * np.sin(np.pi / 1024) ** 2 / (LX / 1024) ** 2
    d = synth.uniform_pm1(15, (nz,))
    ld = np.longdouble
    ref = tridiag.thomas_gth(al.astype(ld), ga.astype(ld), ep.astype(ld), d.astype(ld))
    bnd = tridiag.even_bounds(nz, P)
    x = tridiag.gth_apply(tridiag.gth_prepare(al, ga, ep, bnd), d)
    e_gth = poisson.rel_l2(x, ref)
    a, b, c = tridiag.gth_to_plain(al, ga, ep)
    e_plain = poisson.rel_l2(tridiag.schur_solve(a, b, c, d, bnd), ref)
    assert e_gth < 1e-13
    assert e_plain > 10 * e_gth


def test_gth_prepare_broadcasts_over_columns():
    rng = np.random.default_rng(1)
    n, cols = 24, 7
    al, ga, ep = _random_mmatrix(rng, n, 1e-2)
    shift = rng.random(cols)
    d = rng.standard_normal((n, cols))
    ep2 = ep[:, None] + shift[None, :]
    bnd = tridiag.even_bounds(n, 4)
    x = tridiag.gth_apply(tridiag.gth_prepare(al[:, None] + 0 * ep2, ga[:, None] + 0 * ep2, ep2, bnd), d)
    ref = tridiag.thomas_gth(al[:, None], ga[:, None], ep2, d)
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------- Helmholtz
@pytest.mark.parametrize("bc", [grid.DIRICHLET_CENTRE, grid.DIRICHLET_FACE])
@pytest.mark.parametrize("s", [0.0, 9.615e-9, 1e-3, 10.0])
def test_helmholtz_matches_dense(bc, s):
    nz = 40
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    n = nz if bc == grid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(9, (n, 6, 5))
    u = poisson.solve_helmholtz(r, zf, s, bc)
    ref = dense.helmholtz_dense(r, zf, s, bc)
    assert poisson.rel_l2(u, ref) < 1e-13
    if s == 0.0:
        np.testing.assert_array_equal(u, r)


@pytest.mark.parametrize("bc", [grid.DIRICHLET_CENTRE, grid.DIRICHLET_FACE])
def test_helmholtz_closed_form(bc):
    nz = 32
    zf = synth.tanh_faces(nz, 2.0, 0.0)
    dz = 2.0 / nz
    s = 3e-3
    for m in (1, 2, 7, nz - 1):
        if bc == grid.DIRICHLET_CENTRE:
            v = np.sin(np.pi * m * (np.arange(nz) + 0.5) / nz)
        else:
            v = np.sin(np.pi * m * np.arange(1, nz) / nz)
        mu = -4 * np.sin(np.pi * m / (2 * nz)) ** 2 / dz ** 2
        u = poisson.solve_helmholtz(v[:, None], zf, s, bc)[:, 0]
        np.testing.assert_allclose(u, v / (1 - s * mu), rtol=1e-12, atol=1e-13)


def test_zero_mode_pin_and_consistency():
    nz = 50
    zf = synth.tanh_faces(nz, 2.0, 1.3)
    w = np.diff(zf)
    rhs = synth.uniform_pm1(4, (nz,))
    rhs -= np.dot(w, rhs) / w.sum()
    m = poisson.zero_mode_solve(rhs, zf)
    Lz = dense.lz_dense(zf, dense.NEUMANN)
    np.testing.assert_allclose(Lz @ m, rhs, atol=1e-10 * np.abs(Lz).max() * np.abs(m).max())
    assert abs(np.dot(w, m)) < 1e-14 * np.abs(m).max()


# ------------------------------------------------------- 3-D Helmholtz
@pytest.mark.parametrize("bc", [grid.DIRICHLET_CENTRE, grid.DIRICHLET_FACE])
@pytest.mark.parametrize("nx,ny,nz,beta,s", [(6, 4, 5, 1.5, 1e-2), (7, 5, 6, 2.0, 0.3), (8, 6, 4, 0.0, 5.0)])
def test_helmholtz3d_matches_dense(bc, nx, ny, nz, beta, s):
    zf = synth.tanh_faces(nz, 2.0, beta)
    n = nz if bc == grid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(9, (n, ny, nx))
    got = poisson.solve_helmholtz3d(r, zf, s, bc, LX, LY)
    ref = dense.helmholtz3d_dense(r, zf, s, bc, LX, LY)
    assert poisson.rel_l2(got, ref) < 1e-13


def test_helmholtz3d_reduces_to_columns_for_planar_data():
    # a right-hand side constant in x and y excites only mode (0, 0): the
    # 3-D solve is then the pinned column solve
    nz, s = 12, 0.05
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    col = synth.normal01(4, (nz, 1, 1))
    r = np.broadcast_to(col, (nz, 6, 8)).copy()
    got = poisson.solve_helmholtz3d(r, zf, s, grid.DIRICHLET_CENTRE, LX, LY)
    ref = poisson.solve_helmholtz(col, zf, s, grid.DIRICHLET_CENTRE)
    assert np.max(np.abs(got - ref)) < 1e-13
