"""Linear theory of a perturbed self-gravitating Maxwellian (Sec. 3.2, Eqs. (38)-(40)):
the growth or damping rate of a density mode, and the mode amplitude of a density
field. Reference values for the paper's Tests 2-4; nothing of the numerical method."""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize, special


def growth_root(k_over_kj: float) -> float:
    """y with k^2/k_J^2 = 1 + w Z(w) at w = i y (Eq. (38)); Z(w) = i sqrt(pi) wofz(w)."""
    def h(y):
        w = 1j * y
        return (1 + w * 1j * math.sqrt(math.pi) * special.wofz(w)).real - k_over_kj ** 2
    if k_over_kj < 1:
        return optimize.brentq(h, 1e-9, 1e4, xtol=1e-14)
    return optimize.brentq(h, -5.0, -1e-9, xtol=1e-14)


def gamma_of(k_over_kj: float, G=1.0, rho=1.0) -> float:
    # w = i gamma / (sqrt(8 pi G rho) k/k_J)  (Eq. (40))
    return growth_root(k_over_kj) * math.sqrt(8 * math.pi * G * rho) * k_over_kj


def mode_amplitude(rho, m):
    """|A_m| of delta = rho/mean - 1 along x (Sec. 3.2), for rho of shape (Nx, Ny, Nz)."""
    d = rho / rho.mean() - 1.0
    n = d.shape[0]
    x = np.arange(n)
    return 2 * abs(np.mean(d[:, 0, 0] * np.exp(-2j * np.pi * m * x / n)))
