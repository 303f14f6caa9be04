"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins catch each one: a pin that cannot fail proves nothing."""
import numpy as np
import pytest

import synth
from oracle import dense, grid, poisson, transforms, tridiag

LX, LY = 2 * np.pi, np.pi


def _pin_errors():
    """Largest error of the independent checks used by the pin tests."""
    errs = []
    for (nx, ny, nz, beta) in [(6, 4, 5, 1.5), (7, 5, 6, 2.0)]:
        f, zf = synth.channel_rhs(1, nx, ny, nz, beta=beta)
        errs.append(poisson.rel_l2(poisson.solve_poisson(f, zf, LX, LY),
                                   dense.poisson_dense(f, zf, LX, LY)))
    zf = synth.tanh_faces(12, 2.0, 1.5)
    for bc, n in ((grid.DIRICHLET_CENTRE, 12), (grid.DIRICHLET_FACE, 11)):
        r = synth.normal01(2, (n, 3))
        errs.append(poisson.rel_l2(poisson.solve_helmholtz(r, zf, 1e-2, bc),
                                   dense.helmholtz_dense(r, zf, 1e-2, bc)))
    zf5 = synth.tanh_faces(5, 2.0, 1.5)
    r = synth.normal01(5, (4, 4, 6))                   # w faces: 4 unknowns per column
    errs.append(poisson.rel_l2(poisson.solve_helmholtz3d(r, zf5, 0.2, grid.DIRICHLET_FACE, LX, LY),
                               dense.helmholtz3d_dense(r, zf5, 0.2, grid.DIRICHLET_FACE, LX, LY)))
    for n in (6, 7):
        x = synth.uniform_pm1(n, (n,))
        X = transforms.dft_direct(x)
        P = transforms.rfft_packed(x, axis=0)
        errs.append(abs(P[2] - X[1].real) + abs(P[3] - X[1].imag))
    return max(errs)


def test_unmutated_oracle_passes():
    assert _pin_errors() < 1e-12


def _swap_alpha_gamma(orig):
    def f(zf, bc, dtype=np.float64):
        a, g, e = orig(zf, bc, dtype)
        return np.roll(g, 1), np.roll(a, -1), e
    return f


def _drop_wall_factor(orig):
    def f(zf, bc, dtype=np.float64):
        a, g, e = orig(zf, bc, dtype)
        return a, g, e / 2
    return f


def _wrong_nyquist_slot(orig):
    def f(n, length, dtype=np.float64):
        s = orig(n, length, dtype).copy()
        s[1] = s[2]
        return s
    return f


def _no_pin(orig):
    def f(fhat00, zf):
        m = orig(fhat00, zf)
        return m + 0.1
    return f


def _swapped_re_im(orig):
    def f(x, axis):
        P = np.moveaxis(orig(x, axis), axis, -1).copy()
        P[..., 2], P[..., 3] = P[..., 3].copy(), P[..., 2].copy()
        return np.moveaxis(P, -1, axis)
    return f


def _dropped_forward_term(orig):
    def f(alpha, gamma, eps, d):
        return orig(0 * np.asarray(alpha), gamma, eps + alpha, d)
    return f


@pytest.mark.parametrize("target,attr,mut", [
    (grid, "zop", _swap_alpha_gamma),
    (grid, "zop", _drop_wall_factor),
    (grid, "modified_wavenumbers", _wrong_nyquist_slot),
    (poisson, "zero_mode_solve", _no_pin),
    (transforms, "rfft_packed", _swapped_re_im),
    (tridiag, "thomas_gth", _dropped_forward_term),
])
def test_planted_mistake_is_caught(monkeypatch, target, attr, mut):
    monkeypatch.setattr(target, attr, mut(getattr(target, attr)))
    assert _pin_errors() > 1e-6


# ------------------------------------------------------------ projection
from oracle import projection  # noqa: E402


def _projection_pin_errors():
    """Largest error of the projection pins: D G = L7, a divergence-free
    result, and the removal of a pure gradient field."""
    nx, ny, nz = 8, 6, 7
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    phi = synth.uniform_pm1(31, (nz, ny, nx))
    gx, gy, gz = projection.gradient(phi, zf, LX, LY)
    ref = poisson.apply_L7(phi, zf, LX, LY)
    errs = [np.max(np.abs(projection.divergence(gx, gy, gz, zf, LX, LY) - ref)) / np.max(np.abs(ref))]
    u = synth.uniform_pm1(32, (nz, ny, nx))
    v = synth.uniform_pm1(33, (nz, ny, nx))
    w = synth.uniform_pm1(34, (nz - 1, ny, nx))
    d0 = np.abs(projection.divergence(u, v, w, zf, LX, LY)).max()
    u1, v1, w1, _, _ = projection.project(u, v, w, np.zeros_like(u), zf, LX, LY, gdt=0.3)
    errs.append(np.abs(projection.divergence(u1, v1, w1, zf, LX, LY)).max() / d0)
    u1, v1, w1, _, _ = projection.project(gx, gy, gz, np.zeros_like(u), zf, LX, LY, gdt=0.3)
    errs.append(max(np.abs(x).max() for x in (u1, v1, w1)) / np.abs(gx).max())
    return max(errs)


def test_unmutated_projection_passes():
    assert _projection_pin_errors() < 1e-10


def _div_with_centre_distances(orig):
    def f(u, v, w, zf, lx, ly, *rest):
        zf = np.asarray(zf)
        zc = (zf[1:] + zf[:-1]) / 2
        fake = np.concatenate([[zf[0]], zc[:-1] + np.diff(zc) / 2, [zf[-1]]])
        fake[1:-1] = zf[1:-1] + 0.25 * (np.diff(zc))    # cell widths no longer dzf
        return orig(u, v, w, fake, lx, ly, *rest)
    return f


def _backward_x_gradient(orig):
    def f(phi, zf, lx, ly, *rest):
        gx, gy, gz = orig(phi, zf, lx, ly, *rest)
        return np.roll(gx, 1, axis=2), gy, gz
    return f


def _swapped_w_faces(orig):
    def f(u, v, w, zf, lx, ly, *rest):
        return orig(u, v, -w, zf, lx, ly, *rest)
    return f


def _correction_without_gdt(orig):
    def f(u, v, w, p, zf, lx, ly, gdt, c=0.0, *rest):
        u1, v1, w1, p1, phi = orig(u, v, w, p, zf, lx, ly, gdt, c, *rest)
        return u + (u1 - u) / gdt, v + (v1 - v) / gdt, w + (w1 - w) / gdt, p1, phi
    return f


@pytest.mark.parametrize("attr,mut", [
    ("divergence", _div_with_centre_distances),
    ("gradient", _backward_x_gradient),
    ("divergence", _swapped_w_faces),
    ("project", _correction_without_gdt),
])
def test_planted_projection_mistake_is_caught(monkeypatch, attr, mut):
    monkeypatch.setattr(projection, attr, mut(getattr(projection, attr)))
    assert _projection_pin_errors() > 1e-6


# ------------------------------------------------------------- y walls

def _ywall_pin_errors():
    """Largest error of the y-wall pins: the dense brute force of both wall
    kinds and the even/odd-extension DFTs."""
    errs = []
    for ybc, dybc in ((grid.Y_WALLS, 1), (grid.Y_DIRICHLET, 2)):
        for (nx, ny, nz, beta) in [(4, 5, 6, 1.5), (2, 6, 5, 0.5)]:
            zf = synth.tanh_faces(nz, 2.0, beta)
            f = synth.uniform_pm1(70 + ny, (nz, ny, nx))
            errs.append(poisson.rel_l2(poisson.solve_poisson(f, zf, LX, LY, ybc=ybc),
                                       dense.poisson_dense(f, zf, LX, LY, ybc=dybc)))
    n = 7
    x = synth.uniform_pm1(80, (n,))
    q = np.arange(n)
    E = transforms.dft_direct(np.concatenate([x, x[::-1]]))
    errs.append(np.max(np.abs(transforms.dct2(x, axis=0) - E[:n] * np.exp(-1j * np.pi * q / (2 * n)))))
    O = transforms.dft_direct(np.concatenate([x, -x[::-1]]))
    errs.append(np.max(np.abs(transforms.dst2(x, axis=0)
                              - 1j * np.exp(-1j * np.pi * (q + 1) / (2 * n)) * O[1:n + 1])))
    return max(errs)


def test_unmutated_ywall_oracle_passes():
    assert _ywall_pin_errors() < 1e-12


def _periodic_wavenumbers_for_walls(orig):
    def f(n, length, dtype=np.float64):
        q = np.arange(n, dtype=dtype)
        dx = dtype(length) / n
        return 4 * np.sin(np.pi * q / n) ** 2 / (dx * dx)     # pi q / n instead of pi q / 2n
    return f


def _cosine_phase_off_by_half(orig):
    def f(x, axis):
        x = np.moveaxis(np.asarray(x), axis, -1)
        n = x.shape[-1]
        t = np.arange(n)
        M = 2.0 * np.cos(np.pi * np.outer(t, 2 * t) / (2 * n))   # 2t instead of 2t + 1
        return np.moveaxis(x @ M.T, -1, axis)
    return f


def _sine_modes_from_zero(orig):
    def f(n, length, dtype=np.float64):
        return np.roll(orig(n, length, dtype), 1)                # sigma_{q-1} for mode q
    return f


def _wall_ghost_not_negated(orig):
    def f(n, h, value_zero=False):
        return orig(n, h, False)
    return f


@pytest.mark.parametrize("target,attr,mut", [
    (grid, "wall_wavenumbers", _periodic_wavenumbers_for_walls),
    (transforms, "dct2", _cosine_phase_off_by_half),
    (grid, "dirichlet_wall_wavenumbers", _sine_modes_from_zero),
    (dense, "wall_d2", _wall_ghost_not_negated),
])
def test_planted_ywall_mistake_is_caught(monkeypatch, target, attr, mut):
    monkeypatch.setattr(target, attr, mut(getattr(target, attr)))
    assert _ywall_pin_errors() > 1e-6


# ------------------------------------------------------------- y faces

def _yface_pin_errors():
    """Largest error of the y-face pins: the dense brute force of the 3-D
    Helmholtz on the faces and the odd-extension DFT of the type-I sine
    transform."""
    errs = []
    for bc, n in ((grid.DIRICHLET_CENTRE, 5), (grid.DIRICHLET_FACE, 4)):
        zf = synth.tanh_faces(5, 2.0, 1.5)
        r = synth.uniform_pm1(90 + bc, (n, 6, 4))
        errs.append(poisson.rel_l2(poisson.solve_helmholtz3d(r, zf, 0.05, bc, LX, LY, ybc=grid.Y_FACES),
                                   dense.helmholtz3d_dense(r, zf, 0.05, bc, LX, LY, ybc=3)))
    n = 7
    x = synth.uniform_pm1(95, (n,))
    E = transforms.dft_direct(np.concatenate([[0], x[: n - 1], [0], -x[: n - 1][::-1]]))
    errs.append(np.max(np.abs(transforms.dst1(x, axis=0)[: n - 1] - 1j * E[1:n])))
    return max(errs)


def test_unmutated_yface_oracle_passes():
    assert _yface_pin_errors() < 1e-12


def _face_modes_from_zero(orig):
    def f(n, length, dtype=np.float64):
        return np.roll(orig(n, length, dtype), 1)                # sigma_{q-1} for mode q
    return f


def _face_sine_over_n_plus_one(orig):
    def f(x, axis):
        x = np.moveaxis(np.asarray(x), axis, -1)
        n = x.shape[-1]
        m = np.arange(1, n)
        M = np.zeros((n, n))
        M[: n - 1, : n - 1] = 2.0 * np.sin(np.pi * np.outer(m, m) / (n + 1))   # n + 1 for n
        return np.moveaxis(x @ M.T, -1, axis)
    return f


def _face_inverse_without_scale(orig):
    def f(X, axis):
        return orig(X, axis) * X.shape[axis] / (X.shape[axis] - 1)            # 1/(n-1) for 1/n
    return f


@pytest.mark.parametrize("target,attr,mut", [
    (grid, "face_wall_wavenumbers", _face_modes_from_zero),
    (transforms, "dst1", _face_sine_over_n_plus_one),
    (transforms, "idst1", _face_inverse_without_scale),
])
def test_planted_yface_mistake_is_caught(monkeypatch, target, attr, mut):
    monkeypatch.setattr(target, attr, mut(getattr(target, attr)))
    assert _yface_pin_errors() > 1e-6


# ------------------------------------------------- projection with x walls

def _xwall_projection_pin_errors():
    """D G = L7 with zero-gradient x walls, a divergence-free result, and the
    east wall face's velocity left as it was."""
    nx, ny, nz = 8, 6, 7
    zf = synth.tanh_faces(nz, 2.0, 1.5)
    phi = synth.uniform_pm1(41, (nz, ny, nx))
    gx, gy, gz = projection.gradient(phi, zf, LX, LY, grid.Y_PERIODIC, grid.X_WALLS)
    ref = poisson.apply_L7(phi, zf, LX, LY, grid.Y_PERIODIC, grid.X_WALLS)
    dg = projection.divergence(gx, gy, gz, zf, LX, LY, grid.Y_PERIODIC, grid.X_WALLS)
    errs = [np.max(np.abs(dg - ref)) / np.max(np.abs(ref))]
    u = synth.uniform_pm1(42, (nz, ny, nx))
    v = synth.uniform_pm1(43, (nz, ny, nx))
    w = synth.uniform_pm1(44, (nz - 1, ny, nx))
    d0 = np.abs(projection.divergence(u, v, w, zf, LX, LY, grid.Y_PERIODIC, grid.X_WALLS)).max()
    u1, v1, w1, _, _ = projection.project(u, v, w, np.zeros_like(u), zf, LX, LY, gdt=0.3,
                                          xbc=grid.X_WALLS)
    errs.append(np.abs(projection.divergence(u1, v1, w1, zf, LX, LY, grid.Y_PERIODIC,
                                             grid.X_WALLS)).max() / d0)
    errs.append(np.abs(u1[:, :, -1] - u[:, :, -1]).max())
    return max(errs)


def test_unmutated_xwall_projection_passes():
    assert _xwall_projection_pin_errors() < 1e-10


def _east_wall_flux_kept(orig):
    def f(u, v, w, zf, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
        d = orig(u, v, w, zf, lx, ly, ybc, xbc)
        if xbc == grid.X_WALLS:                        # the wall face's flux counted
            d[:, :, -1] += u[:, :, -1] / (lx / u.shape[2])
        return d
    return f


def _gradient_across_the_east_wall(orig):
    def f(phi, zf, lx, ly, ybc=grid.Y_PERIODIC, xbc=grid.X_PERIODIC):
        return orig(phi, zf, lx, ly, ybc, grid.X_PERIODIC)
    return f


@pytest.mark.parametrize("attr,mut", [
    ("divergence", _east_wall_flux_kept),
    ("gradient", _gradient_across_the_east_wall),
])
def test_planted_xwall_projection_mistake_is_caught(monkeypatch, attr, mut):
    monkeypatch.setattr(projection, attr, mut(getattr(projection, attr)))
    assert _xwall_projection_pin_errors() > 1e-6


def _xface_pin_errors():
    """The dense brute force of the 3-D Helmholtz on the x faces."""
    errs = []
    for bc, n in ((grid.DIRICHLET_CENTRE, 5), (grid.DIRICHLET_FACE, 4)):
        zf = synth.tanh_faces(5, 2.0, 1.5)
        r = synth.uniform_pm1(130 + bc, (n, 4, 6))
        errs.append(poisson.rel_l2(poisson.solve_helmholtz3d(r, zf, 0.05, bc, LX, LY, xbc=grid.X_FACES),
                                   dense.helmholtz3d_dense(r, zf, 0.05, bc, LX, LY, xbc=3)))
    return max(errs)


def test_unmutated_xface_oracle_passes():
    assert _xface_pin_errors() < 1e-12


def _x_faces_as_cell_centres(orig):
    def f(xbc):
        return orig(grid.X_DIRICHLET if xbc == grid.X_FACES else xbc)
    return f


@pytest.mark.parametrize("target,attr,mut", [
    (grid, "face_wall_wavenumbers", _face_modes_from_zero),
    (poisson, "_x_transform", _x_faces_as_cell_centres),
])
def test_planted_xface_mistake_is_caught(monkeypatch, target, attr, mut):
    monkeypatch.setattr(target, attr, mut(getattr(target, attr)))
    assert _xface_pin_errors() > 1e-6
