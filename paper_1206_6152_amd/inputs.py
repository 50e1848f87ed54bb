"""Seeded synthetic initial conditions and workload definitions.

This module generates inputs only; it contains none of the integrator's
arithmetic (no advection, moment, Poisson or acceleration step). Both the GPU
path and the CPU oracle take their inputs from here.

Initial conditions are point values at cell centres, as the paper does for its
King-sphere set-up (Sec. 3.5). A distribution function that is a product of a
spatial factor and a velocity factor is returned as those two factors, so that
large cases can be formed on the device chunk by chunk.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    """Grid, physical constants and run length of one synthetic workload."""
    name: str
    n: tuple                      # spatial cells (Nx, Ny, Nz)
    nv: tuple                     # velocity cells (Nvx, Nvy, Nvz)
    L: tuple                      # box lengths; space is [-L/2, L/2)
    vmin: tuple
    vmax: tuple
    G: float = 1.0
    bc: int = 0                   # 0 periodic, 1 isolated (outflow space)
    dt: float = 0.0               # fixed step used for parity runs
    steps: int = 1
    params: dict = field(default_factory=dict)

    @property
    def shape(self):
        return tuple(self.n) + tuple(self.nv)

    @property
    def cells(self) -> int:
        return int(np.prod(self.n)) * int(np.prod(self.nv))

    def dx(self, l):
        return self.L[l] / self.n[l]

    def dv(self, l):
        return (self.vmax[l] - self.vmin[l]) / self.nv[l]

    def xc(self, l):
        """cell-centre coordinates along spatial axis l"""
        return -0.5 * self.L[l] + (np.arange(self.n[l]) + 0.5) * self.dx(l)

    def vc(self, l):
        """cell-centre velocities along velocity axis l"""
        return self.vmin[l] + (np.arange(self.nv[l]) + 0.5) * self.dv(l)

    def with_grid(self, n=None, nv=None, **kw):
        return replace(self, n=tuple(n or self.n), nv=tuple(nv or self.nv), **kw)


def jeans_sigma(k_over_kj: float, k: float, G: float = 1.0, rho0: float = 1.0) -> float:
    """Velocity dispersion giving k/k_J for wavenumber k, with k_J^2 = 4 pi G rho0 / sigma^2."""
    kj = k / k_over_kj
    return math.sqrt(4.0 * math.pi * G * rho0) / kj


def _cube(name, n, nv, sigma, vbox, dt, steps, **params):
    return Workload(name=name, n=(n, n, n), nv=(nv, nv, nv), L=(1.0, 1.0, 1.0),
                    vmin=(-vbox,) * 3, vmax=(vbox,) * 3, G=1.0, bc=0, dt=dt, steps=steps,
                    params=dict(sigma=sigma, **params))


def landau_8_16() -> Workload:
    """Gravitational Landau damping: periodic unit cube, G = rho0 = 1, 8^3 x 16^3,
    v in [-5s, 5s]^3, f = (1 + 0.05 cos 2 pi x) M_s(v) with k/k_J = 2, CFL 0.5, 20 steps."""
    s = jeans_sigma(2.0, 2.0 * math.pi)
    dt = 0.5 * (1.0 / 8) / (5 * s)
    return _cube("landau_8x16", 8, 16, s, 5 * s, dt, 20, amp=0.05, mode=(1, 0, 0))


def jeans_32_32() -> Workload:
    """Jeans instability: periodic unit cube, k/k_J = 0.5, A = 0.01 along x, 32^3 x 32^3, 50 steps."""
    s = jeans_sigma(0.5, 2.0 * math.pi)
    dt = 0.5 * (1.0 / 32) / (5 * s)
    return _cube("jeans_32x32", 32, 32, s, 5 * s, dt, 50, amp=0.01, mode=(1, 0, 0))


def jeans_adjoint_16_24() -> Workload:
    """Adjoint workload: Jeans sigma, 16^3 x 24^3, fixed dt, 40 steps, per-cell Gaussian
    density perturbation of rms 1e-3 (seed 6152), checkpoint every 8 steps."""
    s = jeans_sigma(0.5, 2.0 * math.pi)
    dt = 0.5 * (1.0 / 16) / (5 * s)
    return _cube("jeans_adjoint_16x24", 16, 24, s, 5 * s, dt, 40, rms=1e-3, seed=6152, ckpt=8)


def slab_16_64_64x64() -> Workload:
    """One GPU's share of a 64^6 run: slab 16 x 64 x 64 of a unit box with 64 cells per
    side (periodic with the slab's own period in x), 64^3 velocity cells in [-1, 1]^3,
    Maxwellian with k_J = 16 pi (sigma = sqrt(4 pi)/(16 pi)) times (1 + delta), delta a
    Gaussian random field with P(k) ~ k^-2, rms 0.02 (seed 1206), 10 steps."""
    s = math.sqrt(4.0 * math.pi) / (16.0 * math.pi)
    return Workload(name="slab_16x64x64_64", n=(16, 64, 64), nv=(64, 64, 64), L=(0.25, 1.0, 1.0),
                    vmin=(-1.0,) * 3, vmax=(1.0,) * 3, G=1.0, bc=0, dt=1.0 / 128, steps=10,
                    params=dict(sigma=s, rms=0.02, index=-2.0, seed=1206))


def white_noise_64_32() -> Workload:
    """Test 4 (Sec. 3.4) in the paper's convergence configuration: periodic unit box,
    64^3 spatial x 32^3 velocity cells, k_J = 16 pi / L (sigma = sqrt(4 pi)/(16 pi)),
    white-noise density, delta uniform in [-0.05, 0.05] per cell (seed 4), to t = 0.8 T.
    Velocity box +-0.5: with it sigma spans 2.26 velocity cells at 32 cells and 4.5
    at 64, the resolution the paper states for this k_J."""
    s = math.sqrt(4.0 * math.pi) / (16.0 * math.pi)
    dt = 0.2 / 13
    return Workload(name="white_noise_64x32", n=(64, 64, 64), nv=(32, 32, 32), L=(1.0, 1.0, 1.0),
                    vmin=(-0.5,) * 3, vmax=(0.5,) * 3, G=1.0, bc=0, dt=dt, steps=52,
                    params=dict(sigma=s, dm=0.1, seed=4, k_jeans=16.0 * math.pi))


def king_48_48(W0: float = 6.0) -> Workload:
    """Isolated King sphere W0 = 6 in units G = sigma = r0 = 1 (so rho0 = 9/(4 pi)):
    box half-width r_t, velocities within the central escape speed sqrt(2 W0),
    48^3 x 48^3, isolated Poisson, 100 steps."""
    model = king_model(W0)
    rt = model.rt
    vesc = math.sqrt(2.0 * W0)
    return Workload(name="king_w6_48x48", n=(48,) * 3, nv=(48,) * 3, L=(2 * rt,) * 3,
                    vmin=(-vesc,) * 3, vmax=(vesc,) * 3, G=1.0, bc=1, dt=0.0, steps=100,
                    params=dict(W0=W0))


def king_units(W0: float):
    """(M, V, T) of one King sphere in units G = sigma = r0 = 1: its mass, V = r0/T and
    T = (G M / r0^3)^(-1/2) (Sec. 3.5)."""
    M = king_model(W0).mass * 9.0 / (4.0 * math.pi)
    T = 1.0 / math.sqrt(M)
    return M, 1.0 / T, T


def king_w3_64x32() -> Workload:
    """Test 5 (Sec. 3.5): King sphere W = 3 in units G = sigma = r0 = 1, box +-5.4 r0,
    velocities +-1.5 V, 64^3 x 32^3 cells, isolated, to t = 1.2 T; the mass is
    renormalised so that 2K/|U| = 1 on the grid."""
    _, V, T = king_units(3.0)
    return Workload(name="king_w3_64x32", n=(64,) * 3, nv=(32,) * 3, L=(10.8,) * 3,
                    vmin=(-1.5 * V,) * 3, vmax=(1.5 * V,) * 3, G=1.0, bc=1, dt=0.0, steps=0,
                    params=dict(W0=3.0, T=T, V=V, spheres=(((0.0, 0.0, 0.0), (0.0, 0.0, 0.0)),)))


def king_merger_64x32() -> Workload:
    """Test 6 (Sec. 3.6), Vlasov side: two W = 3 King spheres at (r0, r0, 0) and
    (-r0, -r0, 0) moving at -0.2 V and +0.2 V along x, box +-6.4 r0, velocities +-2 V,
    64^3 x 32^3 cells, isolated, to t = 5 T."""
    _, V, T = king_units(3.0)
    return Workload(name="king_merger_64x32", n=(64,) * 3, nv=(32,) * 3, L=(12.8,) * 3,
                    vmin=(-2.0 * V,) * 3, vmax=(2.0 * V,) * 3, G=1.0, bc=1, dt=0.0, steps=0,
                    params=dict(W0=3.0, T=T, V=V,
                                spheres=(((1.0, 1.0, 0.0), (-0.2 * V, 0.0, 0.0)),
                                         ((-1.0, -1.0, 0.0), (0.2 * V, 0.0, 0.0)))))


def king_sphere_fields(w: Workload):
    """Per sphere (centre, bulk velocity): Psi/sigma^2 at the spatial cell centres
    (from the sphere's centre) and the cell-centre velocities relative to its bulk
    velocity, for building f = sum of King distribution functions on the device."""
    model = king_model(w.params["W0"])
    X = np.meshgrid(*[w.xc(l) for l in range(3)], indexing="ij")
    out = []
    for c, u in w.params["spheres"]:
        r = np.sqrt(sum((X[l] - c[l]) ** 2 for l in range(3)))
        vrel = [w.vc(l) - u[l] for l in range(3)]
        out.append((model.W_at(r), vrel))
    return out


WORKLOADS = {
    "landau_8x16": landau_8_16,
    "jeans_32x32": jeans_32_32,
    "king_w6_48x48": king_48_48,
    "slab_16x64x64_64": slab_16_64_64x64,
    "jeans_adjoint_16x24": jeans_adjoint_16_24,
    "white_noise_64x32": white_noise_64_32,
    "king_w3_64x32": king_w3_64x32,
    "king_merger_64x32": king_merger_64x32,
}


# ---------------------------------------------------------------------------
# separable Maxwellian initial conditions (Sec. 3.2, 3.4)
# ---------------------------------------------------------------------------

def maxwellian(w: Workload, sigma: float, drift=(0.0, 0.0, 0.0)) -> np.ndarray:
    """M(v) = (2 pi s^2)^(-d/2) exp(-|v - drift|^2 / 2 s^2) at cell-centre velocities,
    over the axes that have more than one velocity cell (a single-cell axis is a
    degenerate dimension of a lower-dimensional test and carries a factor 1/dv)."""
    out = np.ones(tuple(w.nv), dtype=np.float64)
    for l in range(3):
        if w.nv[l] > 1:
            v = w.vc(l) - drift[l]
            g = np.exp(-v * v / (2 * sigma * sigma)) / math.sqrt(2 * math.pi * sigma * sigma)
        else:
            g = np.full(1, 1.0 / w.dv(l))
        shape = [1, 1, 1]
        shape[l] = w.nv[l]
        out = out * g.reshape(shape)
    return out


def cosine_density(w: Workload, rho0: float, amp: float, mode=(1, 0, 0)) -> np.ndarray:
    """rho0 (1 + A cos(k . x)) at cell centres, k = 2 pi mode / L."""
    X = np.meshgrid(*[w.xc(l) for l in range(3)], indexing="ij")
    phase = sum(2 * math.pi * mode[l] * X[l] / w.L[l] for l in range(3))
    return rho0 * (1.0 + amp * np.cos(phase))


def gaussian_random_field(n, L, index: float, rms: float, seed: int) -> np.ndarray:
    """Zero-mean periodic Gaussian random field with power spectrum P(k) ~ k^index,
    normalised to the given rms (numpy default_rng(seed))."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal(tuple(n))
    wk = np.fft.fftn(white)
    ks = np.meshgrid(*[2 * math.pi * np.fft.fftfreq(n[l], d=L[l] / n[l]) for l in range(3)], indexing="ij")
    k2 = ks[0] ** 2 + ks[1] ** 2 + ks[2] ** 2
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (index / 4.0)
    field_ = np.real(np.fft.ifftn(wk * amp))
    field_ -= field_.mean()
    return field_ * (rms / np.sqrt(np.mean(field_ ** 2)))


def gaussian_cells(n, rms: float, seed: int) -> np.ndarray:
    """Independent N(0, rms^2) value per spatial cell (numpy default_rng(seed))."""
    return np.random.default_rng(seed).normal(0.0, rms, size=tuple(n))


def uniform_cells(n, dm: float, seed: int) -> np.ndarray:
    """Independent uniform values in [-dm/2, dm/2] per spatial cell (numpy default_rng(seed)):
    a white-noise density contrast (Sec. 3.4)."""
    return np.random.default_rng(seed).uniform(-0.5 * dm, 0.5 * dm, size=tuple(n))


def separable_factors(w: Workload):
    """(spatial factor [Nx,Ny,Nz], velocity factor [Nvx,Nvy,Nvz]) with f = s (x) m."""
    p = w.params
    s = p["sigma"]
    m = maxwellian(w, s)
    if w.name.startswith("slab"):
        dens = 1.0 + gaussian_random_field(w.n, w.L, p["index"], p["rms"], p["seed"])
    elif w.name.startswith("jeans_adjoint"):
        dens = 1.0 + gaussian_cells(w.n, p["rms"], p["seed"])
    elif w.name.startswith("white_noise"):
        dens = 1.0 + uniform_cells(w.n, p["dm"], p["seed"])
    else:
        dens = cosine_density(w, 1.0, p["amp"], p.get("mode", (1, 0, 0)))
    return dens, m


def initial_f(w: Workload) -> np.ndarray:
    """Full f0 in FP64 (for workloads small enough to hold on the host)."""
    if w.bc == 1:
        return king_f(w)
    dens, m = separable_factors(w)
    return dens.reshape(dens.shape + (1, 1, 1)) * m.reshape((1, 1, 1) + m.shape)


# ---------------------------------------------------------------------------
# King sphere (Sec. 3.5)
# ---------------------------------------------------------------------------

def king_density_shape(W):
    """rho(W)/rho_1 of the King distribution function (Binney & Tremaine eq. 4.114a)."""
    W = np.maximum(np.asarray(W, dtype=np.float64), 0.0)
    from scipy.special import erf
    return np.exp(W) * erf(np.sqrt(W)) - np.sqrt(4 * W / math.pi) * (1 + 2 * W / 3)


@dataclass
class KingModel:
    W0: float
    r: np.ndarray      # radii in units of r0
    W: np.ndarray      # Psi / sigma^2
    rt: float          # tidal radius / r0
    mass: float        # total mass / (rho0 r0^3)

    def W_at(self, radius):
        radius = np.asarray(radius, dtype=np.float64)
        return np.where(radius < self.rt, np.interp(radius, self.r, self.W), 0.0)


def king_model(W0: float, rmax: float = 200.0) -> KingModel:
    """Integrate the King-model Poisson equation outward from W(0) = W0, W'(0) = 0 in
    units r0 = 3 sigma / sqrt(4 pi G rho0): W'' + 2 W'/r = -9 rho(W)/rho0, until W = 0."""
    from scipy.integrate import solve_ivp
    rho_c = float(king_density_shape(W0))

    def rhs(r, y):
        W, dW = y
        src = -9.0 * float(king_density_shape(W)) / rho_c
        if r == 0.0:
            return [dW, src / 3.0]
        return [dW, src - 2.0 * dW / r]

    def edge(r, y):
        return y[0]
    edge.terminal = True
    edge.direction = -1
    r0 = 1e-6
    y0 = [W0 - 1.5 * r0 * r0, -3.0 * r0]
    sol = solve_ivp(rhs, (r0, rmax), y0, events=edge, rtol=1e-11, atol=1e-13, dense_output=True,
                    max_step=0.01)
    rt = float(sol.t_events[0][0])
    r = np.linspace(0.0, rt, 20001)
    W = np.maximum(sol.sol(np.maximum(r, r0))[0], 0.0)
    W[0] = W0
    # mass from the outer boundary: M = -r^2 dW/dr * sigma^2 / G at r_t, in rho0 r0^3 units
    dWt = float(sol.sol(rt)[1])
    mass = -(rt * rt) * dWt * (4 * math.pi / 9.0)
    return KingModel(W0=W0, r=r, W=W, rt=rt, mass=mass)


def king_f(w: Workload, scale: float = 1.0) -> np.ndarray:
    """King distribution function f = rho1 (2 pi sigma^2)^(-3/2) (exp(E/sigma^2) - 1) for
    relative energy E = Psi(r) - v^2/2 > 0, zero otherwise, at cell centres, sigma = 1."""
    W0 = w.params["W0"]
    model = king_model(W0)
    rho0 = 9.0 / (4.0 * math.pi)
    rho1 = rho0 / float(king_density_shape(W0))
    X = np.meshgrid(*[w.xc(l) for l in range(3)], indexing="ij")
    Psi = model.W_at(np.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2))
    V = np.meshgrid(*[w.vc(l) for l in range(3)], indexing="ij")
    v2 = V[0] ** 2 + V[1] ** 2 + V[2] ** 2
    E = Psi.reshape(Psi.shape + (1, 1, 1)) - 0.5 * v2.reshape((1, 1, 1) + v2.shape)
    pref = rho1 * (2 * math.pi) ** -1.5 * scale
    return np.where(E > 0, pref * np.expm1(np.maximum(E, 0.0)), 0.0)


def king_spheres_f(w: Workload, scale: float = 1.0) -> np.ndarray:
    """Sum over the workload's spheres (centre c, bulk velocity u) of the King
    distribution function with E = Psi(|x - c|) - |v - u|^2 / 2, at cell centres, on
    the host in FP64 (for grids small enough to hold there), times scale."""
    pref = king_prefactor(w.params["W0"]) * scale
    f = np.zeros(w.shape, dtype=np.float64)
    for psi, vrel in king_sphere_fields(w):
        V = np.meshgrid(*vrel, indexing="ij")
        hv2 = 0.5 * (V[0] ** 2 + V[1] ** 2 + V[2] ** 2)
        E = psi.reshape(psi.shape + (1, 1, 1)) - hv2.reshape((1, 1, 1) + hv2.shape)
        f += np.where(E > 0, pref * np.expm1(np.maximum(E, 0.0)), 0.0)
    return f


def king_psi(w: Workload) -> np.ndarray:
    """Psi(x)/sigma^2 at spatial cell centres (0 outside the tidal radius)."""
    model = king_model(w.params["W0"])
    X = np.meshgrid(*[w.xc(l) for l in range(3)], indexing="ij")
    return model.W_at(np.sqrt(X[0] ** 2 + X[1] ** 2 + X[2] ** 2))


def king_prefactor(W0: float) -> float:
    rho0 = 9.0 / (4.0 * math.pi)
    return rho0 / float(king_density_shape(W0)) * (2 * math.pi) ** -1.5


# ---------------------------------------------------------------------------
# one-dimensional tests through degenerate axes (Sec. 3.1-3.3)
# ---------------------------------------------------------------------------

def one_d(nx: int, nvx: int, L: float, vbox: float, G: float = 1.0, dt: float = 0.0,
          steps: int = 1, **params) -> Workload:
    """1D-1V phase space as a 6D grid with one cell on the other four axes; the
    single velocity cells span [-1/2, 1/2] so that dv_y dv_z = 1 and v_y = v_z = 0."""
    return Workload(name="one_d", n=(nx, 1, 1), nv=(nvx, 1, 1), L=(L, 1.0, 1.0),
                    vmin=(-vbox, -0.5, -0.5), vmax=(vbox, 0.5, 0.5), G=G, bc=0, dt=dt,
                    steps=steps, params=dict(params))


def random_lines(nlines: int, n: int, seed: int, kind: str = "mixed") -> np.ndarray:
    """Nonnegative test lines: smooth bumps, steps, spikes and noise (default_rng(seed))."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    out = np.empty((nlines, n))
    for i in range(nlines):
        k = kind if kind != "mixed" else ["smooth", "step", "spike", "noise", "sparse"][i % 5]
        if k == "smooth":
            c, w_ = rng.uniform(0.2, 0.8), rng.uniform(0.05, 0.3)
            out[i] = np.exp(-((x - c) / w_) ** 2)
        elif k == "step":
            a, b = np.sort(rng.uniform(0, 1, 2))
            out[i] = ((x > a) & (x < b)).astype(float) * rng.uniform(0.5, 2)
        elif k == "spike":
            out[i] = 0.0
            out[i, rng.integers(0, n)] = rng.uniform(0.5, 2)
        elif k == "noise":
            out[i] = rng.uniform(0, 1, n)
        else:
            out[i] = rng.uniform(0, 1, n) * (rng.uniform(0, 1, n) < 0.3)
    return out
