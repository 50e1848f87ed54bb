"""Pins of the oracle's reverse mode (gradient of the final field energy) against
finite differences of the oracle's forward map and against exact transposes:
the line update (in f and in the Courant number), a velocity sweep including
its dependence on the acceleration, the linear density -> potential ->
acceleration map (dot-product identity), and the full multi-step gradient."""
import numpy as np
import pytest

import oracle
from helpers import oracle_grid, structured_f
from paper_1206_6152_amd import inputs


def _fd_line(f, nu, periodic, lam, df, h):
    plus = oracle.line(f + h * df, nu, periodic)
    minus = oracle.line(f - h * df, nu, periodic)
    return float(lam @ (plus - minus)) / (2 * h)


@pytest.mark.parametrize("periodic", [True, False])
def test_line_vjp_matches_finite_differences(orc, periodic):
    rng = np.random.default_rng(31)
    for t in range(60):
        n = 16
        # generic data: a small jitter breaks exact ties (plateaus at the line
        # maximum, equal neighbours), where the map has kinks and no derivative
        f = inputs.random_lines(1, n, seed=100 + t, kind=["smooth", "noise", "step"][t % 3])[0] + 0.05
        f = f + 1e-3 * rng.uniform(0, 1, n)
        nu = rng.uniform(-2.7, 2.7)
        lam = rng.standard_normal(n)
        df = rng.standard_normal(n)
        lf, dnu = oracle.line_vjp(f, nu, periodic, lam)
        fd = _fd_line(f, nu, periodic, lam, df, 1e-7)
        assert float(lf @ df) == pytest.approx(fd, rel=1e-5, abs=1e-7)
        h = 1e-7
        fdn = float(lam @ (oracle.line(f, nu + h, periodic) - oracle.line(f, nu - h, periodic))) / (2 * h)
        assert dnu == pytest.approx(fdn, rel=1e-5, abs=1e-7)


def test_line_vjp_of_exact_shift_is_the_reverse_shift(orc):
    f = np.abs(np.random.default_rng(2).standard_normal(12)) + 0.1
    lam = np.random.default_rng(3).standard_normal(12)
    lf, _ = oracle.line_vjp(f, 3.0, True, lam)
    np.testing.assert_allclose(lf, np.roll(lam, -3), rtol=1e-14)


@pytest.mark.parametrize("bc", [0, 1])
def test_accel_transpose_dot_product(orc, bc):
    # <lam_a, A f> = <A^T lam_a, f>: A = gradient o potential o density is linear
    w = inputs.Workload(name="t", n=(4, 3, 2), nv=(3, 2, 2), L=(1.0, 0.75, 0.5), vmin=(-1, -1, -1),
                        vmax=(1, 1, 1), G=1.3, bc=bc)
    g = oracle_grid(w)
    rng = np.random.default_rng(7)
    f = rng.uniform(0, 1, w.shape)
    lam_a = rng.standard_normal((3,) + w.n)
    lhs = float(np.sum(lam_a * oracle.accel(g, f)))
    rhs = float(np.sum(oracle.accel_vjp(g, lam_a) * f))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_velocity_sweep_vjp_including_acceleration(orc):
    w = inputs.Workload(name="t", n=(2, 2, 3), nv=(6, 4, 8), L=(1.0, 1.0, 1.5), vmin=(-1, -1, -1),
                        vmax=(1, 1, 1), G=1.0, bc=0)
    g = oracle_grid(w)
    rng = np.random.default_rng(8)
    f = structured_f(w.shape, 9) + 0.01 + 1e-3 * rng.uniform(0, 1, w.shape)   # no exact ties
    tau = 0.3
    a = rng.uniform(-1, 1, (3,) + w.n) * 1.5 * w.dv(0) / tau
    lam = rng.standard_normal(w.shape)
    for axis in (3, 4, 5):
        lf, la = oracle.sweep_vjp(g, f, axis, tau, lam, a)
        df = rng.standard_normal(w.shape)
        da = rng.standard_normal((3,) + w.n) * 1e-1
        h = 1e-7
        plus = oracle.sweep(g, f + h * df, axis, tau, a + h * da)
        minus = oracle.sweep(g, f - h * df, axis, tau, a - h * da)
        fd = float(np.sum(lam * (plus - minus))) / (2 * h)
        an = float(np.sum(lf * df)) + float(np.sum(la * da))
        assert an == pytest.approx(fd, rel=2e-5), axis


@pytest.mark.parametrize("bc", [0, 1])
def test_full_gradient_matches_finite_differences(orc, bc):
    if bc == 0:
        s = inputs.jeans_sigma(0.5, 2 * np.pi)
        w = inputs.Workload(name="t", n=(4, 2, 2), nv=(8, 4, 4), L=(1.0, 0.5, 0.5), vmin=(-4 * s,) * 3,
                            vmax=(4 * s,) * 3, G=1.0, bc=0, dt=0.04, steps=3, params=dict(sigma=s, amp=0.1))
        f0 = inputs.initial_f(w)
        f0 *= 1 + 0.05 * np.random.default_rng(4).standard_normal(w.n).reshape(w.n + (1, 1, 1))
    else:
        # a smooth self-gravitating blob in an isolated box (outflow sweeps)
        w = inputs.Workload(name="t", n=(4, 4, 4), nv=(6, 6, 6), L=(4.0, 4.0, 4.0), vmin=(-2.0,) * 3,
                            vmax=(2.0,) * 3, G=1.0, bc=1, dt=0.2, steps=2, params=dict(sigma=0.6))
        X = np.meshgrid(*[w.xc(l) for l in range(3)], indexing="ij")
        dens = np.exp(-(X[0] ** 2 + X[1] ** 2 + X[2] ** 2) / 2.0)
        f0 = dens.reshape(w.n + (1, 1, 1)) * inputs.maxwellian(w, 0.6).reshape((1, 1, 1) + w.nv)
    # the map is piecewise smooth (corrector branches, line maxima): jitter the
    # data off exact ties and keep the difference step well inside one piece
    f0 = f0 + 1e-6 * f0.max() * np.random.default_rng(9).uniform(0, 1, f0.shape)
    g = oracle_grid(w)
    L, grad = oracle.grad(g, f0, w.steps, w.dt)
    assert L == pytest.approx(oracle.run_loss(g, f0, w.steps, w.dt), rel=1e-14)
    rng = np.random.default_rng(5)
    for t in range(3):
        d = rng.standard_normal(w.shape) * f0.max() * 1e-2
        h = 1e-8   # larger steps cross corrector kinks, smaller ones drown in rounding
        fd = (oracle.run_loss(g, f0 + h * d, w.steps, w.dt) - oracle.run_loss(g, f0 - h * d, w.steps, w.dt)) / (2 * h)
        an = float(np.sum(grad * d))
        assert an == pytest.approx(fd, rel=2e-5), (t, an, fd)
