"""Checks of the synthetic-input generators (not of the integrator): the King
model ODE against an independent fixed-step integrator and its small-radius
series, virial equilibrium of the continuum model, the random fields' stated
statistics, and the separable Maxwellian's normalisation."""
import math

import numpy as np
import pytest

from paper_1206_6152_amd import inputs


def _rk4_king(W0, h=2e-4):
    """independent fixed-step RK4 of W'' + 2W'/r = -9 rho(W)/rho(W0), W(0)=W0, W'(0)=0"""
    rc = float(inputs.king_density_shape(W0))
    def rhs(r, y):
        src = -9.0 * float(inputs.king_density_shape(y[0])) / rc
        return np.array([y[1], src / 3.0 if r == 0 else src - 2 * y[1] / r])
    r, y = 0.0, np.array([W0, 0.0])
    while y[0] > 0:
        k1 = rhs(r, y); k2 = rhs(r + h / 2, y + h / 2 * k1)
        k3 = rhs(r + h / 2, y + h / 2 * k2); k4 = rhs(r + h, y + h * k3)
        y_new = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if y_new[0] <= 0:
            return r + h * y[0] / (y[0] - y_new[0])
        r, y = r + h, y_new
    return r


@pytest.mark.parametrize("W0,rt_expected", [(3.0, 4.699), (6.0, 17.99)])
def test_king_tidal_radius(W0, rt_expected):
    m = inputs.king_model(W0)
    assert m.rt == pytest.approx(rt_expected, rel=2e-3)
    if W0 == 3.0:
        assert m.rt == pytest.approx(_rk4_king(W0, h=1e-3), rel=1e-4)


def test_king_small_radius_series():
    # W = W0 - (9/6) r^2 + ... in units r0 = 3 sigma / sqrt(4 pi G rho0)
    m = inputs.king_model(6.0)
    r = np.array([0.01, 0.02, 0.04])
    np.testing.assert_allclose(m.W_at(r), 6.0 - 1.5 * r * r, rtol=1e-5)


def test_king_mass_two_ways():
    # mass from the boundary slope equals the integral of rho 4 pi r^2
    m = inputs.king_model(6.0)
    rho = inputs.king_density_shape(m.W) / float(inputs.king_density_shape(6.0))
    integral = np.trapezoid(4 * math.pi * m.r ** 2 * rho, m.r)
    assert integral == pytest.approx(m.mass, rel=1e-5)
    assert m.mass == pytest.approx(16.91, rel=2e-3)


def test_gaussian_random_field_statistics():
    d = inputs.gaussian_random_field((16, 64, 64), (0.25, 1.0, 1.0), -2.0, 0.02, 1206)
    assert abs(d.mean()) < 1e-15
    assert np.sqrt(np.mean(d ** 2)) == pytest.approx(0.02, rel=1e-12)
    d2 = inputs.gaussian_random_field((16, 64, 64), (0.25, 1.0, 1.0), -2.0, 0.02, 1206)
    assert np.array_equal(d, d2)


def test_maxwellian_normalisation():
    w = inputs.jeans_32_32()
    m = inputs.maxwellian(w, w.params["sigma"])
    dv3 = w.dv(0) * w.dv(1) * w.dv(2)
    assert m.sum() * dv3 == pytest.approx(1.0, rel=2e-5)


def test_one_d_degenerate_axes():
    w = inputs.one_d(16, 8, L=1.0, vbox=1.0)
    m = inputs.maxwellian(w, 0.3)
    assert m.shape == (8, 1, 1)
    assert w.dv(1) * w.dv(2) == 1.0
    assert w.vc(1)[0] == 0.0 and w.vc(2)[0] == 0.0
