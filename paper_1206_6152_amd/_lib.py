"""ctypes binding of libvp.so (include/vp.h): argument marshalling only.

Every function here has the name of the C entry point it calls. Device memory
and the stream come from PyTorch tensors (their data pointers) and from
``torch.cuda.current_stream()``; all arithmetic runs in the library's HIP
kernels. There is no fallback: if the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvp.so")

VP_OK = 0
VP_EINVAL = -1
VP_ENOMEM = -2
VP_EHIP = -3
VP_ENONFINITE = -4
VP_EUNSUPPORTED = -5
VP_BC_PERIODIC = 0
VP_BC_ISOLATED = 1
VP_F32 = 0
VP_F64 = 1

ERROR_NAMES = {VP_EINVAL: "VP_EINVAL", VP_ENOMEM: "VP_ENOMEM", VP_EHIP: "VP_EHIP",
               VP_ENONFINITE: "VP_ENONFINITE", VP_EUNSUPPORTED: "VP_EUNSUPPORTED"}

# every symbol include/vp.h declares
EXPORTS = ["vp_config_size", "vp_config_validate", "vp_init", "vp_step", "vp_run", "vp_sweep",
           "vp_kick", "vp_drift",
           "vp_accel", "vp_get_accel", "vp_set_accel", "vp_density", "vp_moment", "vp_potential", "vp_energy",
           "vp_dt", "vp_profile_enable", "vp_profile_read", "vp_sweep_adjoint", "vp_kick_adjoint", "vp_accel_adjoint",
           "vp_grad", "vp_stream_copy", "vp_cell_self_integral", "vp_sweep_adjoint_noalloc", "vp_free",
           "vp_last_error"]
VP_NOALLOC_MAX_LINES = 4194304
VP_NPHASE = 14
PHASES = ["x", "y", "z", "vx", "vy", "vz", "gravity", "kick", "kick2", "drift_yz", "adjoint_sweep",
          "adjoint_gravity", "kick_pair", "adjoint_kick"]


class VPError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "VP_E?"), code, message))
        self.code = code


class vp_config(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("nv", ctypes.c_int32 * 3),
        ("L", ctypes.c_double * 3),
        ("vmin", ctypes.c_double * 3),
        ("vmax", ctypes.c_double * 3),
        ("G", ctypes.c_double),
        ("bc", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lock = threading.Lock()
_lib = None


def lib():
    """Load libvp.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvp.so is not built (%s); run paper_1206_6152_amd/build.py "
                               "or __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        C = ctypes.POINTER(vp_config)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        i32, f64 = ctypes.c_int32, ctypes.c_double
        sig = {
            "vp_config_size": [],
            "vp_config_validate": [C],
            "vp_init": [C, P, P, ctypes.POINTER(P)],
            "vp_step": [P, f64],
            "vp_run": [P, i32, f64],
            "vp_sweep": [P, i32, f64],
            "vp_kick": [P, f64],
            "vp_drift": [P, f64],
            "vp_accel": [P],
            "vp_get_accel": [P, P],
            "vp_set_accel": [P, P],
            "vp_density": [P, P],
            "vp_moment": [P, P, P, f64, P],
            "vp_potential": [P, P],
            "vp_energy": [P, D],
            "vp_dt": [P, f64, D],
            "vp_profile_enable": [P, i32],
            "vp_profile_read": [P, D, ctypes.POINTER(ctypes.c_int64)],
            "vp_sweep_adjoint": [P, i32, f64, P, P, P],
            "vp_kick_adjoint": [P, f64, P, P, P],
            "vp_sweep_adjoint_noalloc": [P, i32, f64, P, P, P],
            "vp_accel_adjoint": [P, P, P],
            "vp_grad": [P, i32, f64, i32, P, D],
            "vp_stream_copy": [P, P, ctypes.c_int64, P],
            "vp_free": [P],
            "vp_last_error": [],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.vp_last_error.restype = ctypes.c_char_p
        L.vp_cell_self_integral.argtypes = [f64, f64, f64]
        L.vp_cell_self_integral.restype = f64
        if L.vp_config_size() != ctypes.sizeof(vp_config):
            raise RuntimeError("vp_config layout mismatch between libvp.so and the binding")
        _lib = L
        return L


def check(code: int) -> None:
    if code != VP_OK:
        msg = lib().vp_last_error()
        raise VPError(code, msg.decode() if msg else "")


def make_config(n, nv, L, vmin, vmax, G=1.0, bc=VP_BC_PERIODIC, dtype=VP_F32) -> vp_config:
    c = vp_config()
    for i in range(3):
        c.n[i] = int(n[i])
        c.nv[i] = int(nv[i])
        c.L[i] = float(L[i])
        c.vmin[i] = float(vmin[i])
        c.vmax[i] = float(vmax[i])
    c.G = float(G)
    c.bc = int(bc)
    c.dtype = int(dtype)
    c.flags = 0
    c.reserved = 0
    return c


def vp_config_validate(cfg: vp_config) -> int:
    return lib().vp_config_validate(ctypes.byref(cfg))


def vp_init(cfg: vp_config, f_ptr: int, stream_ptr: int) -> int:
    ctx = ctypes.c_void_p()
    check(lib().vp_init(ctypes.byref(cfg), ctypes.c_void_p(f_ptr), ctypes.c_void_p(stream_ptr),
                        ctypes.byref(ctx)))
    return ctx.value


def vp_step(ctx: int, dt: float) -> None:
    check(lib().vp_step(ctx, float(dt)))


def vp_run(ctx: int, nsteps: int, dt: float) -> None:
    check(lib().vp_run(ctx, int(nsteps), float(dt)))


def vp_sweep(ctx: int, axis: int, tau: float) -> None:
    check(lib().vp_sweep(ctx, int(axis), float(tau)))


def vp_kick(ctx: int, tau: float) -> None:
    check(lib().vp_kick(ctx, float(tau)))


def vp_drift(ctx: int, tau: float) -> None:
    check(lib().vp_drift(ctx, float(tau)))


def vp_accel(ctx: int) -> None:
    check(lib().vp_accel(ctx))


def vp_get_accel(ctx: int, a_ptr: int) -> None:
    check(lib().vp_get_accel(ctx, ctypes.c_void_p(a_ptr)))


def vp_set_accel(ctx: int, a_ptr: int) -> None:
    check(lib().vp_set_accel(ctx, ctypes.c_void_p(a_ptr)))


def vp_density(ctx: int, rho_ptr: int) -> None:
    check(lib().vp_density(ctx, ctypes.c_void_p(rho_ptr)))


def vp_moment(ctx: int, a_ptr: int, w_ptr: int, scale: float, out_ptr: int) -> None:
    check(lib().vp_moment(ctx, ctypes.c_void_p(a_ptr), ctypes.c_void_p(w_ptr), float(scale),
                          ctypes.c_void_p(out_ptr)))


def vp_stream_copy(src_ptr: int, dst_ptr: int, nbytes: int, stream_ptr: int) -> None:
    check(lib().vp_stream_copy(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), ctypes.c_int64(nbytes),
                               ctypes.c_void_p(stream_ptr)))


def vp_cell_self_integral(dx: float, dy: float, dz: float) -> float:
    return float(lib().vp_cell_self_integral(float(dx), float(dy), float(dz)))


def vp_potential(ctx: int, phi_ptr: int) -> None:
    check(lib().vp_potential(ctx, ctypes.c_void_p(phi_ptr)))


def vp_energy(ctx: int):
    out = (ctypes.c_double * 4)()
    check(lib().vp_energy(ctx, out))
    return [out[i] for i in range(4)]


def vp_dt(ctx: int, cfl: float) -> float:
    out = ctypes.c_double()
    check(lib().vp_dt(ctx, float(cfl), ctypes.byref(out)))
    return out.value


def vp_profile_enable(ctx: int, on: bool) -> None:
    check(lib().vp_profile_enable(ctx, 1 if on else 0))


def vp_profile_read(ctx: int):
    """{phase: (total ms, launches)} since profiling was enabled (synchronises)."""
    ms = (ctypes.c_double * VP_NPHASE)()
    n = (ctypes.c_int64 * VP_NPHASE)()
    check(lib().vp_profile_read(ctx, ms, n))
    return {PHASES[i]: (ms[i], n[i]) for i in range(VP_NPHASE)}


def vp_sweep_adjoint(ctx: int, axis: int, tau: float, fin_ptr: int, lam_ptr: int, lam_accel_ptr: int = 0) -> None:
    check(lib().vp_sweep_adjoint(ctx, int(axis), float(tau), ctypes.c_void_p(fin_ptr), ctypes.c_void_p(lam_ptr),
                                 ctypes.c_void_p(lam_accel_ptr or None)))


def vp_kick_adjoint(ctx: int, tau: float, fin_ptr: int, lam_ptr: int, lam_accel_ptr: int = 0) -> None:
    check(lib().vp_kick_adjoint(ctx, float(tau), ctypes.c_void_p(fin_ptr), ctypes.c_void_p(lam_ptr),
                                ctypes.c_void_p(lam_accel_ptr or None)))


def vp_sweep_adjoint_noalloc(ctx: int, axis: int, tau: float, fin_ptr: int, lam_ptr: int,
                             lam_accel_ptr: int = 0) -> None:
    check(lib().vp_sweep_adjoint_noalloc(ctx, int(axis), float(tau), ctypes.c_void_p(fin_ptr),
                                         ctypes.c_void_p(lam_ptr), ctypes.c_void_p(lam_accel_ptr or None)))


def vp_accel_adjoint(ctx: int, lam_accel_ptr: int, lam_ptr: int) -> None:
    check(lib().vp_accel_adjoint(ctx, ctypes.c_void_p(lam_accel_ptr), ctypes.c_void_p(lam_ptr)))


def vp_grad(ctx: int, nsteps: int, dt: float, ckpt_every: int, grad_ptr: int) -> float:
    loss = ctypes.c_double()
    check(lib().vp_grad(ctx, int(nsteps), float(dt), int(ckpt_every), ctypes.c_void_p(grad_ptr), ctypes.byref(loss)))
    return loss.value


def vp_free(ctx: int) -> None:
    if ctx:
        check(lib().vp_free(ctx))


def vp_last_error() -> str:
    m = lib().vp_last_error()
    return m.decode() if m else ""
