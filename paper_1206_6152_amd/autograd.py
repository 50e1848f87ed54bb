"""torch.autograd.Function around the library's reverse mode (vp_grad).

FieldEnergy maps a per-cell initial density perturbation delta(x) to the field
energy L = -U of the final state after a fixed number of steps, for the
initial condition f0(x, v) = rho0 (1 + delta(x)) M(v). Forward and backward
both run in libvp.so: the forward pass and the reverse sweeps (vp_grad), and
the chain rule through that initial-condition map,
dL/d delta(x) = rho0 * sum_v M(v) dL/df0(x, v) (vp_moment). Forming f0 from
delta is input preparation on the device.
"""
from __future__ import annotations

import torch

from . import VP_F32, Simulator, config_of


def initial_f(delta, m_v, rho0: float, dtype):
    """f0 = rho0 (1 + delta) (x) M on the device, formed in FP64 and rounded once."""
    f = (rho0 * (1.0 + delta.double())).reshape(delta.shape + (1, 1, 1)) * m_v.double().reshape((1, 1, 1) + m_v.shape)
    return f.to(dtype).contiguous()


class FieldEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, delta, m_v, workload, vp_dtype, nsteps, dt, ckpt_every, rho0=1.0):
        tdt = torch.float32 if vp_dtype == VP_F32 else torch.float64
        f = initial_f(delta, m_v, rho0, tdt)
        sim = Simulator(config_of(workload, vp_dtype), f)
        loss, g = sim.grad(nsteps, dt, ckpt_every)
        # dL/d delta while the context is at hand (its f is no longer needed)
        gd = sim.moment(g, m_v, rho0)
        sim.close()
        ctx.save_for_backward(gd)
        return torch.tensor(loss, dtype=torch.float64, device=delta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (gd,) = ctx.saved_tensors
        return grad_out * gd, None, None, None, None, None, None, None


def field_energy(delta, m_v, workload, vp_dtype, nsteps, dt, ckpt_every=8, rho0=1.0):
    return FieldEnergy.apply(delta, m_v, workload, vp_dtype, nsteps, dt, ckpt_every, rho0)
