"""MI355X (gfx950) six-dimensional Vlasov-Poisson integrator (PFC scheme).

The compute path is the HIP library ``libvp.so`` behind the C ABI of
``include/vp.h``; this package only marshals arguments to it. ``Simulator``
borrows a torch tensor holding f on the GPU and drives the library on the
current torch stream. Nothing here computes the method itself, and nothing
falls back to the CPU: without the built library every call raises.
"""
from __future__ import annotations

from . import _lib
from ._lib import (VP_BC_ISOLATED, VP_BC_PERIODIC, VP_F32, VP_F64, VPError, make_config,
                   vp_accel, vp_config_validate, vp_density, vp_drift, vp_dt, vp_energy, vp_free, vp_kick,
                   vp_get_accel, vp_init, vp_last_error, vp_potential, vp_profile_enable,
                   vp_profile_read, vp_run, vp_set_accel, vp_step, vp_sweep, vp_sweep_adjoint,
                   vp_kick_adjoint, vp_accel_adjoint, vp_grad, vp_moment)

__all__ = ["Simulator", "VPError", "make_config", "config_of", "VP_F32", "VP_F64",
           "VP_BC_PERIODIC", "VP_BC_ISOLATED", "vp_init", "vp_step", "vp_run", "vp_sweep",
           "vp_kick", "vp_drift",
           "vp_accel", "vp_get_accel", "vp_set_accel", "vp_density", "vp_moment", "vp_potential",
           "vp_energy", "vp_dt", "vp_profile_enable", "vp_profile_read", "vp_sweep_adjoint",
           "vp_accel_adjoint", "vp_grad", "vp_free",
           "vp_last_error", "vp_config_validate"]


def config_of(w, dtype: int = VP_F32):
    """vp_config for a workload description (see ``inputs.Workload``)."""
    return make_config(w.n, w.nv, w.L, w.vmin, w.vmax, G=w.G, bc=w.bc, dtype=dtype)


class Simulator:
    """Owns one library context for a device tensor f of shape (Nx,Ny,Nz,Nvx,Nvy,Nvz).

    f is updated in place by ``step``/``run``/``sweep`` and must stay alive and
    untouched by other code until ``close``.
    """

    def __init__(self, cfg, f):
        import torch
        if not (f.is_cuda and f.is_contiguous()):
            raise ValueError("f must be a contiguous GPU tensor")
        want = torch.float32 if cfg.dtype == VP_F32 else torch.float64
        if f.dtype != want:
            raise ValueError("f dtype %s does not match the configuration" % f.dtype)
        shape = tuple(cfg.n) + tuple(cfg.nv)
        if tuple(f.shape) != shape:
            raise ValueError("f shape %s, expected %s" % (tuple(f.shape), shape))
        self.torch = torch
        self.cfg = cfg
        self.f = f
        self.device = f.device
        self.n = tuple(cfg.n)
        self.stream = torch.cuda.current_stream(f.device)
        self.ctx = vp_init(cfg, f.data_ptr(), self.stream.cuda_stream)

    # -- stepping ----------------------------------------------------------
    def step(self, dt: float):
        vp_step(self.ctx, dt)

    def run(self, nsteps: int, dt: float):
        vp_run(self.ctx, nsteps, dt)

    def sweep(self, axis: int, tau: float):
        vp_sweep(self.ctx, axis, tau)

    def kick(self, tau: float):
        vp_kick(self.ctx, tau)

    def drift(self, tau: float):
        vp_drift(self.ctx, tau)

    def accel(self):
        vp_accel(self.ctx)

    # -- fields --------------------------------------------------------------
    def get_accel(self):
        a = self.torch.empty((3,) + self.n, dtype=self.torch.float64, device=self.device)
        vp_get_accel(self.ctx, a.data_ptr())
        return a

    def set_accel(self, a):
        a = a.to(device=self.device, dtype=self.torch.float64).contiguous()
        assert tuple(a.shape) == (3,) + self.n
        vp_set_accel(self.ctx, a.data_ptr())
        self._keep = a  # keep alive until the async copy has run

    def density(self):
        rho = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        vp_density(self.ctx, rho.data_ptr())
        return rho

    def moment(self, a, w, scale: float = 1.0):
        """scale * sum_v a(x, v) w(v) per spatial cell, FP64 (a like f, w of shape (Nvx, Nvy, Nvz))."""
        w = w.to(device=self.device, dtype=self.torch.float64).contiguous()
        out = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        vp_moment(self.ctx, a.data_ptr(), w.data_ptr(), scale, out.data_ptr())
        return out

    def potential(self):
        phi = self.torch.empty(tuple(x + 2 for x in self.n), dtype=self.torch.float64, device=self.device)
        vp_potential(self.ctx, phi.data_ptr())
        return phi

    def energy(self):
        """[K, U, M, E] (synchronises)"""
        return vp_energy(self.ctx)

    def dt(self, cfl: float) -> float:
        return vp_dt(self.ctx, cfl)

    # -- reverse mode --------------------------------------------------------
    def sweep_adjoint(self, axis: int, tau: float, f_in, lam, lam_accel=None):
        """lam <- J^T lam for T_axis(tau) at forward input f_in (tensors like f)."""
        vp_sweep_adjoint(self.ctx, axis, tau, f_in.data_ptr(), lam.data_ptr(),
                         lam_accel.data_ptr() if lam_accel is not None else 0)

    def kick_adjoint(self, tau: float, f_in, lam, lam_accel=None):
        """lam <- J^T lam for the half kick T_vz T_vy T_vx(tau) at forward input f_in."""
        vp_kick_adjoint(self.ctx, tau, f_in.data_ptr(), lam.data_ptr(),
                        lam_accel.data_ptr() if lam_accel is not None else 0)

    def accel_adjoint(self, lam_accel, lam):
        vp_accel_adjoint(self.ctx, lam_accel.data_ptr(), lam.data_ptr())

    def grad(self, nsteps: int, dt: float, ckpt_every: int = 8):
        """(L, dL/df0) for L = -U after nsteps steps from the current f; f ends at the final state."""
        g = self.torch.empty_like(self.f)
        loss = vp_grad(self.ctx, nsteps, dt, ckpt_every, g.data_ptr())
        return loss, g

    def profile(self, on: bool = True):
        vp_profile_enable(self.ctx, on)

    def profile_read(self):
        return vp_profile_read(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            vp_free(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
