"""FP64 CPU oracle of the six-dimensional Vlasov-Poisson PFC integrator.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. The GPU library neither
imports nor links it, and this package never touches the GPU library.

The arithmetic lives in ``vp_oracle.c`` (plain C, FP64, one routine per
definition in the paper); this module only compiles it with gcc and marshals
numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile vp_oracle.c into liboracle.so (gcc -O2, OpenMP over lines)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class OracleCfg(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("nv", ctypes.c_int32 * 3),
        ("L", ctypes.c_double * 3),
        ("vmin", ctypes.c_double * 3),
        ("vmax", ctypes.c_double * 3),
        ("G", ctypes.c_double),
        ("bc", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            P = ctypes.POINTER(OracleCfg)
            lib.oracle_line.argtypes = [_D, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D]
            lib.oracle_sweep.argtypes = [P, _D, ctypes.c_int, ctypes.c_double, _D]
            lib.oracle_density.argtypes = [P, _D, _D]
            lib.oracle_potential.argtypes = [P, _D, _D]
            lib.oracle_potential_isolated_direct.argtypes = [P, _D, _D]
            lib.oracle_potential_isolated_doubled.argtypes = [P, _D, _D]
            lib.oracle_accel_from_phi.argtypes = [P, _D, _D]
            lib.oracle_accel.argtypes = [P, _D, _D]
            lib.oracle_step.argtypes = [P, _D, ctypes.c_double, _D]
            lib.oracle_dt.argtypes = [P, _D, ctypes.c_double]
            lib.oracle_dt.restype = ctypes.c_double
            lib.oracle_energy.argtypes = [P, _D, _D]
            lib.oracle_cell_self_integral.argtypes = [ctypes.c_double] * 3
            lib.oracle_cell_self_integral.restype = ctypes.c_double
            lib.oracle_num_threads.restype = ctypes.c_int
            lib.oracle_line_vjp.argtypes = [_D, ctypes.c_int, ctypes.c_double, ctypes.c_int, _D, _D]
            lib.oracle_line_vjp.restype = ctypes.c_double
            lib.oracle_sweep_vjp.argtypes = [P, _D, ctypes.c_int, ctypes.c_double, _D, _D, _D]
            lib.oracle_accel_vjp.argtypes = [P, _D, _D]
            lib.oracle_grad.argtypes = [P, _D, ctypes.c_int, ctypes.c_double, _D]
            lib.oracle_grad.restype = ctypes.c_double
            lib.oracle_field_energy_loss.argtypes = [P, _D]
            lib.oracle_field_energy_loss.restype = ctypes.c_double
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


@dataclass
class Grid:
    """Phase-space grid of Sec. 2: space [-L/2, L/2)^3, velocity [vmin, vmax]^3."""
    n: tuple
    nv: tuple
    L: tuple = (1.0, 1.0, 1.0)
    vmin: tuple = (-1.0, -1.0, -1.0)
    vmax: tuple = (1.0, 1.0, 1.0)
    G: float = 1.0
    bc: int = 0  # 0 periodic, 1 isolated/outflow

    def cstruct(self) -> OracleCfg:
        c = OracleCfg()
        for i in range(3):
            c.n[i] = int(self.n[i])
            c.nv[i] = int(self.nv[i])
            c.L[i] = float(self.L[i])
            c.vmin[i] = float(self.vmin[i])
            c.vmax[i] = float(self.vmax[i])
        c.G = float(self.G)
        c.bc = int(self.bc)
        return c

    @property
    def shape(self):
        return tuple(self.n) + tuple(self.nv)

    @property
    def nspace(self):
        return int(np.prod(self.n))

    @property
    def ext_shape(self):
        return tuple(int(x) + 2 for x in self.n)


def line(f, nu: float, periodic: bool, limited: bool = True) -> np.ndarray:
    """One PFC update of a 1D line by nu cells (Sec. 2.1, Eq. (13))."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    lib.oracle_line(_ptr(f), f.size, float(nu), int(periodic), int(limited), _ptr(out))
    return out


def sweep(g: Grid, f: np.ndarray, axis: int, tau: float, accel=None) -> np.ndarray:
    """T_axis(tau) applied to a copy of f (axis 0..5 = x, y, z, vx, vy, vz)."""
    lib = _load()
    out = np.ascontiguousarray(f, dtype=np.float64).copy()
    assert out.shape == g.shape
    c = g.cstruct()
    if axis >= 3:
        a = np.ascontiguousarray(accel, dtype=np.float64).reshape(3, g.nspace)
        lib.oracle_sweep(ctypes.byref(c), _ptr(out), axis, float(tau), _ptr(a))
    else:
        lib.oracle_sweep(ctypes.byref(c), _ptr(out), axis, float(tau), None)
    return out


def density(g: Grid, f: np.ndarray) -> np.ndarray:
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.empty(tuple(g.n), dtype=np.float64)
    c = g.cstruct()
    lib.oracle_density(ctypes.byref(c), _ptr(f), _ptr(rho))
    return rho


def potential(g: Grid, rho: np.ndarray, method: str = "auto") -> np.ndarray:
    """phi with one ghost layer, shape (Nx+2, Ny+2, Nz+2)."""
    lib = _load()
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(tuple(g.n))
    phi = np.zeros(g.ext_shape, dtype=np.float64)
    c = g.cstruct()
    fn = {"auto": lib.oracle_potential, "direct": lib.oracle_potential_isolated_direct,
          "doubled": lib.oracle_potential_isolated_doubled}[method]
    fn(ctypes.byref(c), _ptr(rho), _ptr(phi))
    return phi


def accel_from_phi(g: Grid, phi_ext: np.ndarray) -> np.ndarray:
    lib = _load()
    phi_ext = np.ascontiguousarray(phi_ext, dtype=np.float64)
    a = np.empty((3,) + tuple(g.n), dtype=np.float64)
    c = g.cstruct()
    lib.oracle_accel_from_phi(ctypes.byref(c), _ptr(phi_ext), _ptr(a))
    return a


def accel(g: Grid, f: np.ndarray) -> np.ndarray:
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    a = np.empty((3,) + tuple(g.n), dtype=np.float64)
    c = g.cstruct()
    lib.oracle_accel(ctypes.byref(c), _ptr(f), _ptr(a))
    return a


def step(g: Grid, f: np.ndarray, dt: float, a: np.ndarray) -> None:
    """One step of Eq. (17) in place on f (float64, C-contiguous); a is updated."""
    lib = _load()
    c = g.cstruct()
    lib.oracle_step(ctypes.byref(c), _ptr(f), float(dt), _ptr(a))


def dt(g: Grid, a: np.ndarray, cfl: float) -> float:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    c = g.cstruct()
    return float(lib.oracle_dt(ctypes.byref(c), _ptr(a), float(cfl)))


def energy(g: Grid, f: np.ndarray) -> np.ndarray:
    """[K, U, M, E]."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(4, dtype=np.float64)
    c = g.cstruct()
    lib.oracle_energy(ctypes.byref(c), _ptr(f), _ptr(out))
    return out


def cell_self_integral(dx: float, dy: float, dz: float) -> float:
    return float(_load().oracle_cell_self_integral(dx, dy, dz))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def line_vjp(f, nu: float, periodic: bool, lam_out):
    """(lam_f, dL/dnu) for the line update: lam_f = J^T lam_out."""
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    lo = np.ascontiguousarray(lam_out, dtype=np.float64)
    lf = np.zeros_like(f)
    dnu = lib.oracle_line_vjp(_ptr(f), f.size, float(nu), int(periodic), _ptr(lo), _ptr(lf))
    return lf, float(dnu)


def sweep_vjp(g: Grid, f_in, axis: int, tau: float, lam, accel=None):
    """(J^T lam, lam_accel contribution) of T_axis(tau) at input f_in."""
    lib = _load()
    f_in = np.ascontiguousarray(f_in, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64).copy()
    la = np.zeros((3,) + tuple(g.n))
    c = g.cstruct()
    a = np.ascontiguousarray(accel if accel is not None else np.zeros((3,) + tuple(g.n)), dtype=np.float64)
    lib.oracle_sweep_vjp(ctypes.byref(c), _ptr(f_in), axis, float(tau), _ptr(a), _ptr(lam), _ptr(la))
    return lam, la


def accel_vjp(g: Grid, lam_accel, nv_shape=None):
    """dv3 * (G^T D^T lam_accel) broadcast over velocity, shape of f."""
    lib = _load()
    la = np.ascontiguousarray(lam_accel, dtype=np.float64)
    out = np.zeros(g.shape)
    c = g.cstruct()
    lib.oracle_accel_vjp(ctypes.byref(c), _ptr(la), _ptr(out))
    return out


def grad(g: Grid, f0, nsteps: int, dt_: float):
    """(L, dL/df0) with L = -U after nsteps steps (fixed dt)."""
    lib = _load()
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    out = np.zeros_like(f0)
    c = g.cstruct()
    L = lib.oracle_grad(ctypes.byref(c), _ptr(f0), int(nsteps), float(dt_), _ptr(out))
    return float(L), out


def field_energy_loss(g: Grid, f) -> float:
    lib = _load()
    f = np.ascontiguousarray(f, dtype=np.float64)
    c = g.cstruct()
    return float(lib.oracle_field_energy_loss(ctypes.byref(c), _ptr(f)))


def run_loss(g: Grid, f0, nsteps: int, dt_: float) -> float:
    """L = -U after nsteps steps from f0 (forward only)."""
    r = Run(g, f0)
    for _ in range(nsteps):
        r.step(dt_)
    return field_energy_loss(g, r.f)


@dataclass
class Run:
    """Plain driver: initial acceleration, then steps (reading R5 of vp_oracle.c)."""
    g: Grid
    f: np.ndarray
    a: np.ndarray = field(default=None)

    def __post_init__(self):
        self.f = np.ascontiguousarray(self.f, dtype=np.float64).copy()
        if self.a is None:
            self.a = accel(self.g, self.f)

    def step(self, dt_: float):
        step(self.g, self.f, dt_, self.a)
