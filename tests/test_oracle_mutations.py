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
