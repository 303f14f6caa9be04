"""Pins of the projection oracle (paper Sec. 2.1, eqs. proj1_Lphi,
proj1_ukp1, proj1_Pkp1, proj2_Pkp1) against facts of the staggered-grid
discretisation that do not restate its formulas:

* D G equals the 7-point operator L7 (pinned elsewhere by dense brute force);
* the discrete divergence theorem (periodic x, y; w = 0 on the walls);
* a field built from a stream function is divergence-free and passes the
  projection unchanged; a pure gradient field is removed entirely;
* after a projection the divergence vanishes to rounding;
* the Neumann L_z has the cosine eigenvectors of the uniform grid, which
  fixes the implicit-diffusion pressure update in closed form.
"""
import numpy as np
import pytest

import synth
from oracle import grid, poisson, projection

LX, LY = 2 * np.pi, np.pi


def _fields(seed, nx, ny, nz):
    u = synth.uniform_pm1(seed, (nz, ny, nx))
    v = synth.uniform_pm1(seed + 1, (nz, ny, nx))
    w = synth.uniform_pm1(seed + 2, (nz - 1, ny, nx))
    return u, v, w


@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_div_of_grad_is_the_seven_point_operator(beta):
    nx, ny, nz = 12, 10, 9
    zf = synth.tanh_faces(nz, 2.0, beta)
    phi = synth.uniform_pm1(5, (nz, ny, nx))
    gx, gy, gz = projection.gradient(phi, zf, LX, LY)
    dg = projection.divergence(gx, gy, gz, zf, LX, LY)
    ref = poisson.apply_L7(phi, zf, LX, LY)
    assert np.max(np.abs(dg - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_divergence_theorem():
    nx, ny, nz = 8, 6, 11
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    _, dzf, _ = grid.z_metrics(zf)
    u, v, w = _fields(7, nx, ny, nz)
    d = projection.divergence(u, v, w, zf, LX, LY)
    total = np.dot(dzf, d.reshape(nz, -1).sum(axis=1))
    scale = np.dot(dzf, np.abs(d).reshape(nz, -1).sum(axis=1))
    assert abs(total) <= 1e-14 * scale
    # a flux through one wall face would break it: w on the bottom wall is 0
    w2 = w.copy()
    w2[0] += 1.0
    d2 = projection.divergence(u, v, w2, zf, LX, LY)
    assert np.allclose(d2[0] - d[0], 1.0 / dzf[0])
    assert np.allclose(d2[1] - d[1], -1.0 / dzf[1])


def _stream_field(seed, nx, ny, nz):
    # psi on the cell corners (i+1/2, j+1/2): u = d psi / dy, v = -d psi / dx
    psi = synth.uniform_pm1(seed, (nz, ny, nx))
    dx, dy = LX / nx, LY / ny
    u = (psi - np.roll(psi, 1, axis=1)) / dy
    v = -(psi - np.roll(psi, 1, axis=2)) / dx
    return u, v, np.zeros((nz - 1, ny, nx))


def test_stream_function_field_passes_unchanged():
    nx, ny, nz = 16, 12, 10
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    u, v, w = _stream_field(11, nx, ny, nz)
    assert np.max(np.abs(projection.divergence(u, v, w, zf, LX, LY))) <= 1e-12 * np.max(np.abs(u))
    p = synth.uniform_pm1(12, (nz, ny, nx))
    u1, v1, w1, p1, phi = projection.project(u, v, w, p, zf, LX, LY, gdt=0.37, c=0.0)
    assert np.max(np.abs(phi)) <= 1e-12 * np.max(np.abs(u))
    assert np.max(np.abs(u1 - u)) <= 1e-12 * np.max(np.abs(u))
    assert np.max(np.abs(v1 - v)) <= 1e-12 * np.max(np.abs(v))
    assert np.max(np.abs(p1 - p)) <= 1e-12


def test_gradient_field_is_removed():
    nx, ny, nz = 16, 12, 10
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    psi = synth.uniform_pm1(13, (nz, ny, nx))
    u, v, w = projection.gradient(psi, zf, LX, LY)
    gdt = 0.25
    u1, v1, w1, p1, phi = projection.project(u, v, w, np.zeros_like(u), zf, LX, LY, gdt=gdt)
    big = max(np.max(np.abs(u)), np.max(np.abs(v)), np.max(np.abs(w)))
    for x in (u1, v1, w1):
        assert np.max(np.abs(x)) <= 1e-11 * big
    # phi = psi / gdt up to the constant that pins its weighted mean
    _, dzf, _ = grid.z_metrics(zf)
    d = phi - psi / gdt
    assert np.max(np.abs(d - d.mean())) <= 1e-11 * np.max(np.abs(psi / gdt))


@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_projected_field_is_divergence_free(beta):
    nx, ny, nz = 16, 8, 12
    zf = synth.tanh_faces(nz, 2.0, beta)
    u, v, w = _fields(21, nx, ny, nz)
    d0 = projection.divergence(u, v, w, zf, LX, LY)
    u1, v1, w1, _, _ = projection.project(u, v, w, np.zeros_like(u), zf, LX, LY, gdt=0.1)
    d1 = projection.divergence(u1, v1, w1, zf, LX, LY)
    assert np.sqrt(np.sum(d1 ** 2)) <= 1e-12 * np.sqrt(np.sum(d0 ** 2))


def test_neumann_lz_cosine_eigenvectors_and_pressure_update():
    nz = 16
    zf = synth.tanh_faces(nz, 2.0, 0.0)    # uniform: dz = 2 / nz
    dz = 2.0 / nz
    k = np.arange(nz)
    for m in (0, 1, 5, nz - 1):
        e = np.cos(np.pi * m * (k + 0.5) / nz)
        lam = (2 - 2 * np.cos(np.pi * m / nz)) / dz ** 2
        phi = np.broadcast_to(e[:, None, None], (nz, 2, 4)).copy()
        lz = projection.lz_neumann(phi, zf)
        assert np.allclose(lz, -lam * phi, atol=1e-12 * max(lam, 1.0))
    # through project(): u* = gdt G e (m >= 1 has zero mean), so phi = e and
    # p_new - p_old = e - c L_z e = (1 + c lam) e
    nx, ny, m, gdt, c = 8, 4, 3, 0.2, 0.013
    e = np.cos(np.pi * m * (k + 0.5) / nz)
    lam = (2 - 2 * np.cos(np.pi * m / nz)) / dz ** 2
    phi_e = np.broadcast_to(e[:, None, None], (nz, ny, nx)).copy()
    u, v, w = (gdt * g for g in projection.gradient(phi_e, zf, LX, LY))
    p = synth.uniform_pm1(3, (nz, ny, nx))
    u1, v1, w1, p1, phi = projection.project(u, v, w, p, zf, LX, LY, gdt=gdt, c=c)
    assert np.max(np.abs(phi - phi_e)) <= 1e-12
    assert np.max(np.abs((p1 - p) - (1 + c * lam) * phi_e)) <= 1e-12 * (1 + c * lam)
    assert np.max(np.abs(w1)) <= 1e-12 * np.max(np.abs(w))


# zero-gradient walls at both y ends (v[:, ny-1] is the top wall face)

@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_y_walls_div_of_grad_is_the_seven_point_operator(beta):
    nx, ny, nz = 12, 10, 9
    zf = synth.tanh_faces(nz, 2.0, beta)
    phi = synth.uniform_pm1(55, (nz, ny, nx))
    gx, gy, gz = projection.gradient(phi, zf, LX, LY, grid.Y_WALLS)
    dg = projection.divergence(gx, gy, gz, zf, LX, LY, grid.Y_WALLS)
    ref = poisson.apply_L7(phi, zf, LX, LY, grid.Y_WALLS)
    assert np.max(np.abs(dg - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_y_walls_divergence_theorem_and_projection():
    nx, ny, nz = 8, 6, 11
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    _, dzf, _ = grid.z_metrics(zf)
    u, v, w = _fields(57, nx, ny, nz)
    d = projection.divergence(u, v, w, zf, LX, LY, grid.Y_WALLS)
    total = np.dot(dzf, d.reshape(nz, -1).sum(axis=1))
    assert abs(total) <= 1e-14 * np.dot(dzf, np.abs(d).reshape(nz, -1).sum(axis=1))
    # the top wall face is ignored
    v2 = v.copy()
    v2[:, ny - 1] += 3.0
    assert np.array_equal(projection.divergence(u, v2, w, zf, LX, LY, grid.Y_WALLS), d)
    u1, v1, w1, _, _ = projection.project(u, v, w, np.zeros_like(u), zf, LX, LY, gdt=0.2,
                                          ybc=grid.Y_WALLS)
    d1 = projection.divergence(u1, v1, w1, zf, LX, LY, grid.Y_WALLS)
    assert np.sqrt(np.sum(d1 ** 2)) <= 1e-12 * np.sqrt(np.sum(d ** 2))
    assert np.array_equal(v1[:, ny - 1], v[:, ny - 1])


# zero-gradient walls at both x ends (u[:, :, nx-1] is the east wall face),
# alone and with y walls

@pytest.mark.parametrize("ybc", [grid.Y_PERIODIC, grid.Y_WALLS])
@pytest.mark.parametrize("beta", [0.0, 1.5])
def test_x_walls_div_of_grad_is_the_seven_point_operator(beta, ybc):
    nx, ny, nz = 10, 12, 9
    zf = synth.tanh_faces(nz, 2.0, beta)
    phi = synth.uniform_pm1(58, (nz, ny, nx))
    gx, gy, gz = projection.gradient(phi, zf, LX, LY, ybc, grid.X_WALLS)
    dg = projection.divergence(gx, gy, gz, zf, LX, LY, ybc, grid.X_WALLS)
    ref = poisson.apply_L7(phi, zf, LX, LY, ybc, grid.X_WALLS)
    assert np.max(np.abs(dg - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("ybc", [grid.Y_PERIODIC, grid.Y_WALLS])
def test_x_walls_divergence_theorem_and_projection(ybc):
    nx, ny, nz = 6, 8, 11
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    _, dzf, _ = grid.z_metrics(zf)
    u, v, w = _fields(59, nx, ny, nz)
    d = projection.divergence(u, v, w, zf, LX, LY, ybc, grid.X_WALLS)
    total = np.dot(dzf, d.reshape(nz, -1).sum(axis=1))
    assert abs(total) <= 1e-14 * np.dot(dzf, np.abs(d).reshape(nz, -1).sum(axis=1))
    # the east wall face is ignored
    u2 = u.copy()
    u2[:, :, nx - 1] += 3.0
    assert np.array_equal(projection.divergence(u2, v, w, zf, LX, LY, ybc, grid.X_WALLS), d)
    u1, v1, w1, _, _ = projection.project(u, v, w, np.zeros_like(u), zf, LX, LY, gdt=0.2,
                                          ybc=ybc, xbc=grid.X_WALLS)
    d1 = projection.divergence(u1, v1, w1, zf, LX, LY, ybc, grid.X_WALLS)
    assert np.sqrt(np.sum(d1 ** 2)) <= 1e-12 * np.sqrt(np.sum(d ** 2))
    assert np.array_equal(u1[:, :, nx - 1], u[:, :, nx - 1])
