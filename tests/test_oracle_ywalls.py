"""Pins of the oracle's wall-bounded y direction (paper Sec. 2.2.1: the
cosine and sine members of the Fourier-based transforms, for zero-gradient
and value-zero walls at both y ends), against facts that do not restate its
formulas:

* the cosine (sine) transform equals the even- (odd-) extension DFT of
  length 2n by direct summation, and its inverse undoes it;
* the cosine (sine) vectors are eigenvectors of the dense wall second
  difference (assembled from face fluxes) with the stated wavenumbers;
* the Poisson solve equals the dense least-squares brute force on tiny grids;
* its 7-point residual vanishes at round-off; it is linear, and mirror
  symmetric in y.
"""
import numpy as np
import pytest

import synth
from oracle import dense, grid, poisson, transforms

LX, LY = 2 * np.pi, np.pi


@pytest.mark.parametrize("n", [1, 2, 5, 8, 12])
def test_cosine_transform_is_the_even_extension_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    e = np.concatenate([x, x[::-1]])                       # x_0..x_{n-1}, x_{n-1}..x_0
    E = transforms.dft_direct(e)
    q = np.arange(n)
    # the even extension's DFT is 2 exp(i pi q / 2n) X_q
    ref = E[:n] * np.exp(-1j * np.pi * q / (2 * n))
    X = transforms.dct2(x, axis=0)
    assert np.max(np.abs(X - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(transforms.idct2(X, axis=0) - x)) <= 1e-13 * n


@pytest.mark.parametrize("n", [2, 3, 8, 13])
def test_cosine_vectors_diagonalise_the_wall_second_difference(n):
    h = 0.37
    D = dense.wall_d2(n, h)
    sig = grid.wall_wavenumbers(n, n * h)
    t = np.arange(n)
    for q in range(n):
        e = np.cos(np.pi * q * (2 * t + 1) / (2 * n))
        assert np.max(np.abs(D @ e + sig[q] * e)) <= 1e-10 * max(1.0, sig[q])


@pytest.mark.parametrize("nx,ny,nz,beta,seed", [
    (4, 3, 5, 1.5, 0), (2, 4, 6, 0.0, 1), (6, 5, 4, 2.0, 2), (4, 1, 5, 1.0, 3), (1, 6, 7, 1.2, 4),
])
def test_solve_matches_dense_brute_force(nx, ny, nz, beta, seed):
    zf = synth.tanh_faces(nz, 2.0, beta)
    f = synth.uniform_pm1(seed, (nz, ny, nx))
    got = poisson.solve_poisson(f, zf, LX, LY, ybc=grid.Y_WALLS)
    ref = dense.poisson_dense(f, zf, LX, LY, ybc=1)
    assert np.max(np.abs(got - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_residual_linearity_and_mirror_symmetry():
    nx, ny, nz = 16, 12, 20
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    f = synth.uniform_pm1(7, (nz, ny, nx))
    g = synth.uniform_pm1(8, (nz, ny, nx))
    p = poisson.solve_poisson(f, zf, LX, LY, ybc=grid.Y_WALLS)
    r = poisson.residual7(p, f, zf, LX, LY, ybc=grid.Y_WALLS)
    assert np.max(np.abs(r)) <= 1e-11 * np.max(np.abs(f))
    # the periodic operator would see a different residual: the walls matter
    rp = poisson.residual7(p, f, zf, LX, LY)
    assert np.max(np.abs(rp)) > 1e-3 * np.max(np.abs(f))
    q = poisson.solve_poisson(g, zf, LX, LY, ybc=grid.Y_WALLS)
    pq = poisson.solve_poisson(2 * f - 3 * g, zf, LX, LY, ybc=grid.Y_WALLS)
    assert np.max(np.abs(pq - (2 * p - 3 * q))) <= 1e-11 * np.max(np.abs(pq))
    pm = poisson.solve_poisson(f[:, ::-1].copy(), zf, LX, LY, ybc=grid.Y_WALLS)
    assert np.max(np.abs(pm - p[:, ::-1])) <= 1e-11 * np.max(np.abs(p))


# value-zero (Dirichlet) y walls: the sine transform

@pytest.mark.parametrize("n", [1, 2, 5, 8, 12])
def test_sine_transform_is_the_odd_extension_dft(n):
    rng = np.random.default_rng(40 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    e = np.concatenate([x, -x[::-1]])
    E = transforms.dft_direct(e)
    q = np.arange(1, n + 1)
    # the odd extension's DFT at mode q is -i exp(i pi q / 2n) Y_{q-1}
    ref = 1j * np.exp(-1j * np.pi * q / (2 * n)) * E[1:n + 1]
    Y = transforms.dst2(x, axis=0)
    assert np.max(np.abs(Y - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(transforms.idst2(Y, axis=0) - x)) <= 1e-13 * n


@pytest.mark.parametrize("n", [1, 2, 3, 8, 13])
def test_sine_vectors_diagonalise_the_value_zero_second_difference(n):
    h = 0.29
    D = dense.wall_d2(n, h, value_zero=True)
    sig = grid.dirichlet_wall_wavenumbers(n, n * h)
    t = np.arange(n)
    for q in range(n):
        e = np.sin(np.pi * (q + 1) * (2 * t + 1) / (2 * n))
        assert np.max(np.abs(D @ e + sig[q] * e)) <= 1e-10 * max(1.0, sig[q])


@pytest.mark.parametrize("nx,ny,nz,beta,seed", [
    (4, 3, 5, 1.5, 10), (2, 4, 6, 0.0, 11), (6, 5, 4, 2.0, 12), (4, 1, 5, 1.0, 13),
])
def test_dirichlet_solve_matches_dense_brute_force(nx, ny, nz, beta, seed):
    zf = synth.tanh_faces(nz, 2.0, beta)
    f = synth.uniform_pm1(seed, (nz, ny, nx))
    got = poisson.solve_poisson(f, zf, LX, LY, ybc=grid.Y_DIRICHLET)
    ref = dense.poisson_dense(f, zf, LX, LY, ybc=2)
    assert np.max(np.abs(got - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


def test_dirichlet_residual_and_no_mean_projection():
    nx, ny, nz = 16, 12, 20
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    f = synth.uniform_pm1(17, (nz, ny, nx)) + 0.5     # a non-zero mean stays in the problem
    p = poisson.solve_poisson(f, zf, LX, LY, ybc=grid.Y_DIRICHLET)
    lp = poisson.apply_L7(p, zf, LX, LY, ybc=grid.Y_DIRICHLET)
    assert np.max(np.abs(lp - f)) <= 1e-11 * np.max(np.abs(f))
    pm = poisson.solve_poisson(f[:, ::-1].copy(), zf, LX, LY, ybc=grid.Y_DIRICHLET)
    assert np.max(np.abs(pm - p[:, ::-1])) <= 1e-11 * np.max(np.abs(p))


@pytest.mark.parametrize("ybc,dense_ybc", [(grid.Y_WALLS, 1), (grid.Y_DIRICHLET, 2)])
@pytest.mark.parametrize("bc", [grid.DIRICHLET_CENTRE, grid.DIRICHLET_FACE])
def test_helmholtz3d_with_y_walls_matches_dense(ybc, dense_ybc, bc):
    nx, ny, nz, s = 4, 5, 6, 0.07
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    n = nz if bc == grid.DIRICHLET_CENTRE else nz - 1
    r = synth.uniform_pm1(50 + ybc + 3 * bc, (n, ny, nx))
    got = poisson.solve_helmholtz3d(r, zf, s, bc, LX, LY, ybc=ybc)
    ref = dense.helmholtz3d_dense(r, zf, s, bc, LX, LY, ybc=dense_ybc)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


# a field on the y faces between value-zero walls (the face-located velocity
# of a y-walled grid): the type-I sine transform

@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
def test_type1_sine_transform_is_the_odd_extension_dft(n):
    rng = np.random.default_rng(70 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)   # row n-1: the wall, not read
    f = x[: n - 1]                                              # faces 1..n-1
    e = np.concatenate([[0], f, [0], -f[::-1]])                # odd extension, length 2n
    E = transforms.dft_direct(e)
    # the odd extension's DFT at q is -2i sum_m x_m sin(pi q m / n) = -i X_q
    ref = np.zeros(n, dtype=complex)
    ref[: n - 1] = 1j * E[1:n]
    X = transforms.dst1(x, axis=0)
    assert np.max(np.abs(X - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    back = transforms.idst1(X, axis=0)
    assert np.max(np.abs(back[: n - 1] - f)) <= 1e-13 * n
    assert back[n - 1] == 0


@pytest.mark.parametrize("n", [2, 3, 8, 13])
def test_type1_sine_vectors_diagonalise_the_face_second_difference(n):
    h = 0.31
    D = dense.face_d2(n, h)
    sig = grid.face_wall_wavenumbers(n, n * h)
    m = np.arange(1, n)
    for q in range(1, n):
        e = np.sin(np.pi * q * m / n)
        assert np.max(np.abs(D @ e + sig[q - 1] * e)) <= 1e-10 * max(1.0, sig[q - 1])


@pytest.mark.parametrize("bc", [grid.DIRICHLET_CENTRE, grid.DIRICHLET_FACE])
@pytest.mark.parametrize("xbc,dense_xbc", [(grid.X_PERIODIC, 0), (grid.X_WALLS, 1), (grid.X_DIRICHLET, 2)])
def test_helmholtz3d_on_y_faces_matches_dense(bc, xbc, dense_xbc):
    nx, ny, nz, s = 4, 6, 5, 0.05
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    n = nz if bc == grid.DIRICHLET_CENTRE else nz - 1
    r = synth.uniform_pm1(80 + bc + 3 * dense_xbc, (n, ny, nx))
    got = poisson.solve_helmholtz3d(r, zf, s, bc, LX, LY, ybc=grid.Y_FACES, xbc=xbc)
    ref = dense.helmholtz3d_dense(r, zf, s, bc, LX, LY, ybc=3, xbc=dense_xbc)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.all(got[:, ny - 1, :] == 0)


def test_helmholtz3d_on_y_faces_residual_from_face_fluxes():
    # (I - s L) u = r on the interior faces, L assembled from face-to-face
    # differences with the wall faces at zero, independently of the dense
    # matrices above
    nx, ny, nz, s = 8, 10, 6, 0.03
    zf = synth.tanh_faces(nz, 2.0, 1.2)
    r = synth.uniform_pm1(91, (nz, ny, nx))
    u = poisson.solve_helmholtz3d(r, zf, s, grid.DIRICHLET_CENTRE, LX, LY, ybc=grid.Y_FACES)
    dx, dy = LX / nx, LY / ny
    ui = u[:, : ny - 1, :]
    pad = np.concatenate([np.zeros((nz, 1, nx)), ui, np.zeros((nz, 1, nx))], axis=1)
    lyy = (pad[:, 2:, :] - 2 * ui + pad[:, :-2, :]) / dy ** 2
    lxx = (np.roll(ui, -1, 2) - 2 * ui + np.roll(ui, 1, 2)) / dx ** 2
    al, ga, ex = grid.zop(zf, grid.DIRICHLET_CENTRE)
    lz = -(al + ga + ex)[:, None, None] * ui
    lz[1:] += al[1:, None, None] * ui[:-1]
    lz[:-1] += ga[:-1, None, None] * ui[1:]
    res = r[:, : ny - 1, :] - (ui - s * (lxx + lyy + lz))
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(r))


def test_poisson_rejects_y_faces():
    zf = synth.tanh_faces(4, 2.0, 1.0)
    with pytest.raises(ValueError):
        poisson.solve_poisson(np.zeros((4, 4, 4)), zf, LX, LY, ybc=grid.Y_FACES)
