"""Pins of the oracle's wall-bounded x direction (paper Sec. 2.2.1: the cosine
and sine members of the Fourier-based transforms, here at both x ends; the
transforms themselves are pinned along y in test_oracle_ywalls, and act the
same along any axis), against facts that do not restate its formulas:

* the Poisson solve with walls in x, alone and with walls in y, equals the
  dense least-squares (or, with value-zero walls, dense) brute force on tiny
  grids;
* the 7-point operator with x walls equals the dense flux-form operator;
* the solve is mirror symmetric in x and its residual vanishes at round-off;
* the 3-D Helmholtz with x walls equals its dense solve;
* a planted mistake (the periodic transform with wall wavenumbers) fails.
"""
import numpy as np
import pytest

import synth
from oracle import dense, grid, poisson, transforms

LX, LY = 2 * np.pi, np.pi
XB = {"walls": grid.X_WALLS, "dirichlet": grid.X_DIRICHLET}
YB = {"periodic": grid.Y_PERIODIC, "walls": grid.Y_WALLS, "dirichlet": grid.Y_DIRICHLET}


@pytest.mark.parametrize("xbc", ["walls", "dirichlet"])
@pytest.mark.parametrize("ybc", ["periodic", "walls", "dirichlet"])
@pytest.mark.parametrize("nx,ny,nz,beta,seed", [(4, 3, 5, 1.5, 0), (5, 4, 4, 0.0, 1), (3, 6, 6, 2.0, 2)])
def test_solve_matches_dense_brute_force(nx, ny, nz, beta, seed, xbc, ybc):
    zf = synth.tanh_faces(nz, 2.0, beta)
    f = synth.uniform_pm1(600 + seed, (nz, ny, nx))
    got = poisson.solve_poisson(f, zf, LX, LY, ybc=YB[ybc], xbc=XB[xbc])
    ref = dense.poisson_dense(f, zf, LX, LY, ybc=YB[ybc], xbc=XB[xbc])
    assert np.max(np.abs(got - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("xbc", ["walls", "dirichlet"])
@pytest.mark.parametrize("ybc", ["periodic", "walls"])
def test_operator_matches_dense_flux_form(xbc, ybc):
    nx, ny, nz = 5, 4, 6
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    p = synth.uniform_pm1(610, (nz, ny, nx))
    got = poisson.apply_L7(p, zf, LX, LY, ybc=YB[ybc], xbc=XB[xbc])
    ref = (dense.l7_dense(nx, ny, zf, LX, LY, YB[ybc], XB[xbc]) @ p.reshape(-1)).reshape(p.shape)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("xbc", ["walls", "dirichlet"])
def test_residual_and_mirror_symmetry(xbc):
    nx, ny, nz = 24, 16, 20
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    f = synth.uniform_pm1(620, (nz, ny, nx))
    p = poisson.solve_poisson(f, zf, LX, LY, xbc=XB[xbc])
    r = poisson.residual7(p, f, zf, LX, LY, xbc=XB[xbc])
    assert np.max(np.abs(r)) <= 1e-12 * np.max(np.abs(f))
    pm = poisson.solve_poisson(f[:, :, ::-1].copy(), zf, LX, LY, xbc=XB[xbc])
    assert np.max(np.abs(pm - p[:, :, ::-1])) <= 1e-12 * np.max(np.abs(p))
    # the periodic operator does not annihilate this residual
    rp = poisson.residual7(p, f, zf, LX, LY)
    assert np.max(np.abs(rp)) > 1e-3 * np.max(np.abs(f))


@pytest.mark.parametrize("xbc", ["walls", "dirichlet"])
@pytest.mark.parametrize("bc,dbc", [(grid.DIRICHLET_CENTRE, dense.DIRICHLET_CENTRE),
                                    (grid.DIRICHLET_FACE, dense.DIRICHLET_FACE)])
def test_helmholtz3d_matches_dense(xbc, bc, dbc):
    nx, ny, nz, s = 4, 3, 6, 0.05
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    n = nz if bc == grid.DIRICHLET_CENTRE else nz - 1
    r = synth.normal01(630, (n, ny, nx))
    got = poisson.solve_helmholtz3d(r, zf, s, bc, LX, LY, ybc=grid.Y_WALLS, xbc=XB[xbc])
    ref = dense.helmholtz3d_dense(r, zf, s, dbc, LX, LY, ybc=1, xbc=XB[xbc])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_planted_mistake_is_caught(monkeypatch):
    """The periodic x transform with the wall wavenumbers: not a solution."""
    nx, ny, nz = 4, 3, 5
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    f = synth.uniform_pm1(640, (nz, ny, nx))
    ref = dense.poisson_dense(f, zf, LX, LY, xbc=grid.X_WALLS)
    monkeypatch.setattr(poisson, "_x_transform", lambda xbc: (
        transforms.rfft_packed, transforms.irfft_packed, grid.wall_wavenumbers))
    got = poisson.solve_poisson(f, zf, LX, LY, xbc=grid.X_WALLS)
    assert np.max(np.abs(got - ref)) > 1e-3 * np.max(np.abs(ref))


# a field on the x faces between value-zero walls (the face-located u of an
# x-walled grid): the type-I sine transform along x

@pytest.mark.parametrize("bc", [grid.DIRICHLET_CENTRE, grid.DIRICHLET_FACE])
@pytest.mark.parametrize("ybc,dense_ybc", [(grid.Y_PERIODIC, 0), (grid.Y_WALLS, 1), (grid.Y_FACES, 3)])
def test_helmholtz3d_on_x_faces_matches_dense(bc, ybc, dense_ybc):
    nx, ny, nz, s = 6, 4, 5, 0.05
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    n = nz if bc == grid.DIRICHLET_CENTRE else nz - 1
    r = synth.uniform_pm1(110 + bc + 3 * dense_ybc, (n, ny, nx))
    got = poisson.solve_helmholtz3d(r, zf, s, bc, LX, LY, ybc=ybc, xbc=grid.X_FACES)
    ref = dense.helmholtz3d_dense(r, zf, s, bc, LX, LY, ybc=dense_ybc, xbc=3)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.all(got[:, :, nx - 1] == 0)


def test_helmholtz3d_on_x_faces_residual_from_face_fluxes():
    nx, ny, nz, s = 10, 8, 6, 0.03
    zf = synth.tanh_faces(nz, 2.0, 1.2)
    r = synth.uniform_pm1(121, (nz, ny, nx))
    u = poisson.solve_helmholtz3d(r, zf, s, grid.DIRICHLET_CENTRE, LX, LY, xbc=grid.X_FACES)
    dx, dy = LX / nx, LY / ny
    ui = u[:, :, : nx - 1]
    pad = np.concatenate([np.zeros((nz, ny, 1)), ui, np.zeros((nz, ny, 1))], axis=2)
    lxx = (pad[:, :, 2:] - 2 * ui + pad[:, :, :-2]) / dx ** 2
    lyy = (np.roll(ui, -1, 1) - 2 * ui + np.roll(ui, 1, 1)) / dy ** 2
    al, ga, ex = grid.zop(zf, grid.DIRICHLET_CENTRE)
    lz = -(al + ga + ex)[:, None, None] * ui
    lz[1:] += al[1:, None, None] * ui[:-1]
    lz[:-1] += ga[:-1, None, None] * ui[1:]
    res = r[:, :, : nx - 1] - (ui - s * (lxx + lyy + lz))
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(r))


def test_poisson_rejects_x_faces():
    zf = synth.tanh_faces(4, 2.0, 1.0)
    with pytest.raises(ValueError):
        poisson.solve_poisson(np.zeros((4, 4, 4)), zf, LX, LY, xbc=grid.X_FACES)
