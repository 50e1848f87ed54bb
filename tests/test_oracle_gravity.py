"""Pins of the oracle's gravity (Sec. 2.2) and diagnostics against closed forms:
the discrete Laplacian identity behind Eq. (20), a single Fourier mode, the
plain convolution against the doubled-grid transform (Eq. (21)), a point mass,
the cell self-potential integral, the two-point gradient of Eq. (22), and the
time-step rule of Eqs. (23)-(25)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import Grid


def _lap7(phi_ext, d):
    """7-point Laplacian of the interior of a ghost-padded array"""
    c = phi_ext[1:-1, 1:-1, 1:-1]
    out = np.zeros_like(c)
    for ax in range(3):
        sl_p = [slice(1, -1)] * 3
        sl_m = [slice(1, -1)] * 3
        sl_p[ax] = slice(2, None)
        sl_m[ax] = slice(None, -2)
        out += (phi_ext[tuple(sl_p)] - 2 * c + phi_ext[tuple(sl_m)]) / d[ax] ** 2
    return out


def test_periodic_potential_solves_discrete_poisson(orc):
    # G_hat of Eq. (20) is the inverse of the 7-point Laplacian, so
    # lap7(phi) = 4 pi G (rho - mean rho) for any rho (k = 0 removed).
    g = Grid(n=(8, 6, 4), nv=(1, 1, 1), L=(1.0, 0.7, 0.5), G=1.3)
    rho = np.random.default_rng(3).uniform(0.5, 1.5, g.n)
    phi = orc.potential(g, rho)
    d = [g.L[i] / g.n[i] for i in range(3)]
    np.testing.assert_allclose(_lap7(phi, d), 4 * math.pi * g.G * (rho - rho.mean()), rtol=0, atol=1e-11)
    assert abs(phi[1:-1, 1:-1, 1:-1].mean()) < 1e-13
    # ghosts are periodic images
    np.testing.assert_array_equal(phi[0, 1:-1, 1:-1], phi[-2, 1:-1, 1:-1])
    np.testing.assert_array_equal(phi[-1, 1:-1, 1:-1], phi[1, 1:-1, 1:-1])


def test_periodic_single_mode_closed_form(orc):
    n, m = 16, 3
    g = Grid(n=(n, 1, 1), nv=(1, 1, 1), L=(2.0, 1.0, 1.0), G=0.7)
    dx = g.L[0] / n
    x = -g.L[0] / 2 + (np.arange(n) + 0.5) * dx
    rho = np.cos(2 * np.pi * m * x / g.L[0]).reshape(n, 1, 1)
    phi = orc.potential(g, rho)[1:-1, 1, 1]
    exact = -math.pi * g.G * dx * dx * np.cos(2 * np.pi * m * x / g.L[0]) / math.sin(math.pi * m / n) ** 2
    np.testing.assert_allclose(phi, exact, rtol=0, atol=1e-13)


def test_isolated_direct_sum_equals_doubled_grid(orc):
    g = Grid(n=(6, 5, 4), nv=(1, 1, 1), L=(3.0, 2.5, 2.0), G=1.0, bc=1)
    rho = np.random.default_rng(4).uniform(0, 1, g.n)
    a = orc.potential(g, rho, method="direct")
    b = orc.potential(g, rho, method="doubled")
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-13 * np.abs(a).max())


def test_isolated_point_mass(orc):
    # a single occupied cell: phi = -G m / r exactly away from it, and
    # -G m / (dx dy dz) * (integral of 1/r over the cell) on it.
    g = Grid(n=(7, 7, 7), nv=(1, 1, 1), L=(3.5, 3.5, 3.5), G=2.0, bc=1)
    d = 0.5
    mass = 1.7
    rho = np.zeros(g.n)
    rho[2, 3, 4] = mass / d ** 3
    phi = orc.potential(g, rho, method="direct")
    idx = np.indices(g.ext_shape) - 1
    r = np.sqrt(((idx[0] - 2) * d) ** 2 + ((idx[1] - 3) * d) ** 2 + ((idx[2] - 4) * d) ** 2)
    off = r > 0
    np.testing.assert_allclose(phi[off], -g.G * mass / r[off], rtol=1e-14)
    self_ = phi[3, 4, 5]
    np.testing.assert_allclose(self_, -g.G * mass / d ** 3 * orc.cell_self_integral(d, d, d), rtol=1e-14)


def test_cell_self_integral_by_quadrature(orc):
    # integral of 1/|r| over a centred box, by adaptive quadrature of one octant
    for (a, b, c) in [(1.0, 1.0, 1.0), (1.0, 0.5, 2.0), (0.3, 0.7, 0.4)]:
        val, err = integrate.tplquad(lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z),
                                     0, a / 2, 0, b / 2, 0, c / 2, epsabs=1e-11, epsrel=1e-10)
        np.testing.assert_allclose(orc.cell_self_integral(a, b, c), 8 * val, rtol=1e-8)
    # the unit-cube constant
    np.testing.assert_allclose(orc.cell_self_integral(1, 1, 1), 2.3800773640, rtol=1e-10)


def test_isolated_far_field_is_monopole(orc):
    g = Grid(n=(12, 12, 12), nv=(1, 1, 1), L=(12.0, 12.0, 12.0), G=1.0, bc=1)
    rho = np.zeros(g.n)
    rho[5:7, 5:7, 5:7] = 1.0
    M = rho.sum()
    phi = orc.potential(g, rho)
    # corner ghost cell (-1,-1,-1) is sqrt(3)*6.5 cells from the centre of mass (5.5,5.5,5.5)
    r = math.sqrt(3) * 6.5
    assert abs(phi[0, 0, 0] / (-M / r) - 1) < 2e-3


def test_two_point_gradient_of_mode(orc):
    n = 12
    g = Grid(n=(1, n, 1), nv=(1, 1, 1), L=(1.0, 3.0, 1.0))
    d = 3.0 / n
    k = 2 * np.pi * 2 / 3.0
    y = -1.5 + (np.arange(-1, n + 1) + 0.5) * d
    phi = np.zeros(g.ext_shape)
    phi[:, :, :] = np.cos(k * y).reshape(1, -1, 1)
    a = orc.accel_from_phi(g, phi)
    yc = y[1:-1]
    np.testing.assert_allclose(a[1, 0, :, 0], np.sin(k * yc) * math.sin(k * d) / d, rtol=0, atol=1e-13)
    assert np.all(a[0] == 0) and np.all(a[2] == 0)


def test_density_is_velocity_integral(orc):
    g = Grid(n=(2, 3, 1), nv=(4, 5, 6), vmin=(-1, -2, -3), vmax=(1, 2, 3))
    f = np.random.default_rng(1).uniform(0, 1, g.shape)
    rho = orc.density(g, f)
    dv3 = (2 / 4) * (4 / 5) * (6 / 6)
    np.testing.assert_allclose(rho, f.sum(axis=(3, 4, 5)) * dv3, rtol=1e-14)


def test_energy_of_uniform_maxwellian(orc):
    # midpoint quadrature of a wide Gaussian is spectrally accurate:
    # M = rho L^3, K = (3/2) sigma^2 M, U = 0 for a uniform periodic density
    from paper_1206_6152_amd import inputs
    w = inputs.landau_8_16().with_grid(n=(4, 4, 4), nv=(24, 24, 24))
    g = Grid(n=w.n, nv=w.nv, L=w.L, vmin=w.vmin, vmax=w.vmax, G=w.G)
    s = w.params["sigma"]
    m = inputs.maxwellian(w, s)
    f = np.broadcast_to(m, w.shape).copy()
    K, U, M, E = orc.energy(g, f)
    np.testing.assert_allclose(M, 1.0, rtol=1e-5)
    np.testing.assert_allclose(K, 1.5 * s * s * M, rtol=1e-4)
    assert abs(U) < 1e-14


def test_energy_of_single_mode_potential(orc):
    # U = 1/2 sum rho phi dx^3 with phi from Eq. (20): for rho = rho0 + A cos(kx)
    # on N cells, U = -(A^2 / 4) pi G dx^2 / sin^2(pi m / N) * L^3 (mean removed)
    n, mmode, A = 16, 2, 0.1
    g = Grid(n=(n, 2, 2), nv=(1, 1, 1), L=(1.0, 1.0, 1.0), vmin=(-0.5,) * 3, vmax=(0.5,) * 3, G=1.0)
    x = -0.5 + (np.arange(n) + 0.5) / n
    rho = 1.0 + A * np.cos(2 * np.pi * mmode * x)
    f = np.broadcast_to(rho.reshape(n, 1, 1, 1, 1, 1), g.shape).copy()
    K, U, M, E = orc.energy(g, f)
    dx = 1.0 / n
    exact = -(A * A / 4) * math.pi * dx * dx / math.sin(math.pi * mmode / n) ** 2
    np.testing.assert_allclose(U, exact, rtol=1e-12)
    np.testing.assert_allclose(M, 1.0, rtol=1e-14)


def test_timestep_rule(orc):
    g = Grid(n=(8, 4, 2), nv=(4, 4, 4), L=(1.0, 2.0, 4.0), vmin=(-1, -3, -0.5), vmax=(2, 1, 0.5))
    a = np.zeros((3,) + g.n)
    # dt_p = min(0.125/2, 0.5/3, 2/0.5) = 0.0625; no acceleration -> dt_v = inf
    assert orc.dt(g, a, 0.5) == pytest.approx(0.5 * 0.0625, rel=1e-15)
    a[1, 3, 2, 1] = -40.0   # dv_y = 1 -> 1/40 = 0.025
    a[2, 0, 0, 0] = 10.0    # dv_z = 0.25 -> 0.025
    a[0, 1, 1, 1] = 100.0   # dv_x = 0.75 -> 0.0075
    assert orc.dt(g, a, 0.3) == pytest.approx(0.3 * 0.0075, rel=1e-15)
