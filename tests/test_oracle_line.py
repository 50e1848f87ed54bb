"""Pins of the oracle's one-dimensional PFC operator (Sec. 2.1) against facts the
paper and the mathematics fix: exact translation at integer Courant numbers,
mass conservation, positivity and the maximum principle, third-order accuracy
of the unlimited profile and its exactness on quadratics, and the relation
between the outflow and periodic boundary conditions."""
import numpy as np
import pytest

from paper_1206_6152_amd import inputs


@pytest.mark.parametrize("nu", [-5, -3, -1, 0, 1, 2, 7])
def test_integer_shift_is_exact_translation_periodic(orc, nu):
    # Test 1 (Sec. 3.1): free streaming translates the profile; at integer
    # Courant numbers the traced-back cell is exactly another cell.
    f = inputs.random_lines(10, 32, seed=11).ravel()[:32] + 0.1
    for row in inputs.random_lines(10, 32, seed=12):
        out = orc.line(row, nu, periodic=True)
        assert np.array_equal(out, np.roll(row, nu))
    assert np.array_equal(orc.line(f, nu, True), np.roll(f, nu))


@pytest.mark.parametrize("nu", [-3, -1, 1, 4])
def test_integer_shift_outflow_zero_fill(orc, nu):
    for row in inputs.random_lines(10, 24, seed=13):
        out = orc.line(row, nu, periodic=False)
        ref = np.zeros_like(row)
        if nu > 0:
            ref[nu:] = row[:-nu]
        else:
            ref[:nu] = row[-nu:]
        assert np.array_equal(out, ref)


def test_periodic_conserves_mass(orc):
    rng = np.random.default_rng(5)
    for row in inputs.random_lines(60, 48, seed=14):
        nu = rng.uniform(-3.5, 3.5)
        out = orc.line(row, nu, periodic=True)
        assert abs(out.sum() - row.sum()) <= 1e-13 * row.sum()


def test_outflow_equals_periodic_on_zero_padded_line(orc):
    # Outflow boundaries: matter that leaves is lost and nothing enters
    # (Sec. 2.1). On a line padded with enough empty cells, the periodic update
    # restricted to the original cells must be the outflow update, and the pad
    # receives exactly the mass that left.
    rng = np.random.default_rng(6)
    for row in inputs.random_lines(40, 32, seed=15):
        nu = rng.uniform(-2.9, 2.9)
        pad = 8
        padded = np.concatenate([np.zeros(pad), row, np.zeros(pad)])
        per = orc.line(padded, nu, periodic=True)
        out = orc.line(row, nu, periodic=False)
        np.testing.assert_allclose(out, per[pad:-pad], rtol=0, atol=1e-14 * row.max())
        lost = row.sum() - out.sum()
        np.testing.assert_allclose(lost, per[:pad].sum() + per[-pad:].sum(), rtol=1e-12, atol=1e-13 * row.sum())


@pytest.mark.parametrize("kind", ["step", "spike", "noise", "sparse", "smooth"])
def test_positivity_and_maximum_principle(orc, kind):
    # Sec. 2.1: the scheme preserves positivity and obeys the maximum principle.
    rng = np.random.default_rng(7)
    for row in inputs.random_lines(200, 40, seed=16, kind=kind):
        finf = row.max()
        for nu in rng.uniform(-1.0, 1.0, 3):
            for periodic in (True, False):
                out = orc.line(row, nu, periodic)
                assert out.min() >= -1e-15 * finf
                assert out.max() <= finf * (1 + 1e-14)


def test_unlimited_profile_violates_bounds(orc):
    # Control: without the slope correctors the same data overshoot, so the
    # maximum-principle test above has teeth.
    row = np.zeros(32)
    row[10:20] = 1.0
    out = orc.line(row, 0.5, periodic=True, limited=False)
    assert out.max() > 1.01 or out.min() < -0.01


def _cell_avg(F, x0, x1):
    return (F(x1) - F(x0)) / (x1 - x0)


def test_unlimited_third_order_convergence(orc):
    # "third order approximation" (Sec. 2.1): error of one update on a smooth
    # periodic profile falls as Dx^3.
    errs = []
    sizes = [32, 64, 128, 256]
    nu = 0.37
    for n in sizes:
        dx = 1.0 / n
        edges = np.arange(n + 1) * dx
        F = lambda x: x - np.cos(2 * np.pi * x) / (2 * np.pi) * 0.5  # antiderivative of 1 + 0.5 sin
        f = (F(edges[1:]) - F(edges[:-1])) / dx
        exact = (F(edges[1:] - nu * dx) - F(edges[:-1] - nu * dx)) / dx
        out = orc.line(f, nu, periodic=True, limited=False)
        errs.append(np.abs(out - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 2.85), orders


def test_limited_equals_unlimited_on_well_resolved_positive_profile(orc):
    # Away from the line maximum (where the corrector bounded by f_inf clips the
    # peak) and far above zero, the correctors are 1 and the two profiles agree.
    n = 64
    x = (np.arange(n) + 0.5) / n
    f = 2.0 + 0.3 * np.sin(2 * np.pi * x)
    away = np.abs(np.arange(n) - np.argmax(f)) > 4
    for nu in (-0.8, -0.2, 0.3, 0.9):
        a = orc.line(f, nu, True, limited=True)
        b = orc.line(f, nu, True, limited=False)
        np.testing.assert_allclose(a[away], b[away], rtol=1e-15, atol=0)
        assert np.abs(a - b).max() > 0  # the clip at the peak is real


@pytest.mark.parametrize("nu", [-1.7, -0.6, -0.25, 0.1, 0.5, 0.93, 2.4])
def test_quadratic_cell_averages_advect_exactly(orc, nu):
    # The unlimited profile is the parabola with cell averages f_{i-1}, f_i,
    # f_{i+1}; on cell averages of a global quadratic it is that quadratic, so
    # the update equals the exact average over the traced-back cell. Checked on
    # cells whose stencil stays inside the line.
    n = 40
    # positive and monotone, so neither corrector bound is reached inside
    P = lambda x: 3.0 * x + 0.025 * x * x + 0.001 * x ** 3 / 3.0
    lo = np.arange(n) - 0.5
    f = P(lo + 1) - P(lo)
    out = orc.line(f, nu, periodic=False, limited=False)
    exact = P(lo + 1 - nu) - P(lo - nu)
    m = int(np.ceil(abs(nu))) + 2
    np.testing.assert_allclose(out[m:n - m], exact[m:n - m], rtol=1e-13)
    # and the limiter leaves it alone in the interior
    out_l = orc.line(f, nu, periodic=False, limited=True)
    np.testing.assert_allclose(out_l[m:n - m], exact[m:n - m], rtol=1e-13)


def test_reflection_symmetry(orc):
    # x -> -x with u -> -u maps the problem onto itself.
    rng = np.random.default_rng(8)
    for row in inputs.random_lines(50, 30, seed=17):
        nu = rng.uniform(-2.5, 2.5)
        for periodic in (True, False):
            a = orc.line(row, nu, periodic)
            b = orc.line(row[::-1].copy(), -nu, periodic)[::-1]
            np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-14 * row.max())


def test_constant_line_invariant_periodic(orc):
    f = np.full(16, 0.75)
    for nu in (-2.3, -0.4, 0.0, 0.6, 1.5):
        np.testing.assert_allclose(orc.line(f, nu, True), f, rtol=1e-15)


def test_top_hat_no_oscillation(orc):
    # Test 1 (Sec. 3.1): the sharp edge is transported without oscillation and
    # f stays within [0, 1].
    n = 128
    f = np.zeros(n)
    f[n // 4: 3 * n // 4] = 1.0
    g = f.copy()
    for _ in range(300):
        g = orc.line(g, 0.3, True)
    assert g.min() >= 0.0 and g.max() <= 1.0 + 1e-14
    # monotone on each side of the (smeared) plateau: no new local extrema
    d = np.diff(np.concatenate([g, g[:1]]))
    sign_changes = np.sum(np.abs(np.diff(np.sign(d[np.abs(d) > 1e-12]))) > 0)
    assert sign_changes <= 2
    assert abs(g.sum() - f.sum()) < 1e-11


def test_single_cell_lines(orc):
    f = np.array([0.4])
    np.testing.assert_allclose(orc.line(f, 0.3, True), f, rtol=1e-15)
    np.testing.assert_allclose(orc.line(f, 0.0, False), f, rtol=0)
    # outflow: a single cell loses the fraction nu of a flat profile
    np.testing.assert_allclose(orc.line(f, 0.3, False), [0.4 * 0.7], rtol=1e-15)


def _steep_cases():
    # Cell averages of a parabola whose one-sided differences sit between one
    # and two times the distance to the bound the corrector guards (Sec. 2.1,
    # slope corrector of the PFC scheme). With the corrector's factor 2 the
    # parabola is left exact on those cells; a factor 1 would cut the slope.
    #   rise:  q(x) = (x - s)^2 on cells centred at integers right of the
    #          minimum (eps+ against 2 f): for s = 0 the cell at 2 has
    #          D+/f = 5/(4 + 1/12) = 1.22; for s = -1/2 the cell centred at
    #          1.5 has D+/f = 4/(2.25 + 1/12) = 1.71.
    #   fall:  the mirror image, left of the minimum (eps- against 2 f).
    #   cap:   q(x) = A - x^2, line maximum f_inf = A - 1/12 at cell 0. The
    #          cell at -2 has D-/(f_inf - f) = 5/4 (eps- against f_inf) and the
    #          cell at +2 has |D+|/(f_inf - f) = 5/4 (eps+ against f_inf).
    cases = []
    for s in (0.0, -0.5):
        P = lambda x, s=s: (x - s) ** 3 / 3.0
        cases.append(("rise", P, np.arange(0, 24) + 0.0))
        P = lambda x, s=s: (x + s) ** 3 / 3.0
        cases.append(("fall", P, np.arange(-23, 1) + 0.0))
    A = 50.0
    P = lambda x: A * x - x ** 3 / 3.0
    cases.append(("cap", P, np.arange(-6, 7) + 0.0))
    return cases


def _used_cells(i, nu):
    # cells whose profile the update of cell i integrates over
    a, b = i - 0.5 - nu, i + 0.5 - nu
    return set(range(int(np.floor(a + 0.5)), int(np.floor(b + 0.5)) + 1))


@pytest.mark.parametrize("nu", [-1.6, -0.7, -0.3, 0.2, 0.55, 0.85, 1.4])
def test_steep_quadratic_cell_averages_advect_exactly_under_the_correctors(orc, nu):
    hit = 0
    branches = set()
    for kind, P, centres in _steep_cases():
        f = P(centres + 0.5) - P(centres - 0.5)
        assert f.min() > 0.0
        finf = f.max()
        # the corrector each difference meets and the bound it is held to
        bounds = []
        for k in range(len(f)):
            row = {}
            if k + 1 < len(f):
                d = f[k + 1] - f[k]
                row["+"] = (abs(d), 2 * f[k] if d > 0 else 2 * (finf - f[k]), "eps+ f" if d > 0 else "eps+ finf")
            if k > 0:
                d = f[k] - f[k - 1]
                row["-"] = (abs(d), 2 * (finf - f[k]) if d > 0 else 2 * f[k], "eps- finf" if d > 0 else "eps- f")
            bounds.append(row)
        # unlimited with the factor 2: every difference within its bound
        exact_ok = np.array([len(b) == 2 and all(d <= bd for d, bd, _ in b.values()) for b in bounds])
        # steep: unlimited with the factor 2, limited with a factor 1
        steep_j = [k for k, b in enumerate(bounds)
                   if exact_ok[k] and any(d > 0.5 * bd for d, bd, _ in b.values())]
        assert steep_j, kind
        out = orc.line(f, nu, periodic=False, limited=True)
        exact = (P(centres + 0.5 - nu) - P(centres - 0.5 - nu))
        for i in range(len(f)):
            used = _used_cells(i, nu)
            if not all(0 <= k < len(f) and exact_ok[k] for k in used):
                continue
            np.testing.assert_allclose(out[i], exact[i], rtol=1e-13, err_msg="%s cell %d" % (kind, i))
            for k in used & set(steep_j):
                hit += 1
                branches.update(name for d, bd, name in bounds[k].values() if d > 0.5 * bd)
    # updates that read a steep cell were checked, for each of the four bounds
    assert hit >= 5
    assert branches == {"eps+ f", "eps+ finf", "eps- f", "eps- finf"}
