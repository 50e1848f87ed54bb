"""GPU checks of the two halves of Eq. (17) through the C ABI: vp_kick (the
three velocity sweeps, one pass over f when the velocity block fits on chip)
and vp_drift (the three position sweeps) must equal the corresponding single
vp_sweep calls bit for bit, and the oracle within the parity tolerances."""
import numpy as np
import pytest

import oracle
from helpers import oracle_grid, rel_l1, small_workload, structured_f
from paper_1206_6152_amd import VP_BC_ISOLATED, VP_BC_PERIODIC, VP_F32, VP_F64, Simulator, config_of

pytestmark = pytest.mark.gpu

NP = {VP_F64: np.float64, VP_F32: np.float32}


def _sim(w, f0, dtype, accel):
    import torch
    f = torch.from_numpy(np.ascontiguousarray(f0.astype(NP[dtype]))).to("cuda:0")
    sim = Simulator(config_of(w, dtype), f)
    sim.set_accel(torch.from_numpy(np.ascontiguousarray(accel)))
    return sim, f


def _accel(w, nu_max, tau, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (3,) + tuple(w.n))
    for l in range(3):
        a[l] *= nu_max * w.dv(l) / abs(tau)
    return a


CASES = [(VP_F32, 8), (VP_F32, 16), (VP_F32, 24), (VP_F32, 32), (VP_F64, 8), (VP_F64, 16),
         (VP_F64, 24), (VP_F64, 32)]


@pytest.mark.parametrize("dtype,nv", CASES)
@pytest.mark.parametrize("nu_max", [0.45, 1.7])
def test_kick_equals_three_sweeps_and_oracle(dtype, nv, nu_max):
    print("case", dtype, nv, nu_max, flush=True)
    w = small_workload(VP_BC_PERIODIC, n=(3, 2, 4), nv=(nv, nv, nv))
    f0 = structured_f(w.shape, seed=nv).astype(NP[dtype]).astype(np.float64)
    tau = 0.41
    a = _accel(w, nu_max, tau, seed=nv + 1)
    sim, f = _sim(w, f0, dtype, a)
    sim.kick(tau)
    fused = f.cpu().numpy()
    sim.close()
    sim, f = _sim(w, f0, dtype, a)
    for ax in (3, 4, 5):
        sim.sweep(ax, tau)
    split = f.cpu().numpy()
    sim.close()
    assert np.array_equal(fused, split)
    g = oracle_grid(w)
    ref = f0
    for ax in (3, 4, 5):
        ref = oracle.sweep(g, ref, ax, tau, a)
    tol = 1e-14 if dtype == VP_F64 else 2e-6
    assert rel_l1(fused, ref) <= tol


@pytest.mark.parametrize("dtype", [VP_F32, VP_F64])
def test_kick_non_cubic_velocity_grid_falls_back(dtype):
    w = small_workload(VP_BC_PERIODIC, n=(2, 2, 3), nv=(8, 12, 16))
    f0 = structured_f(w.shape, seed=4).astype(NP[dtype]).astype(np.float64)
    a = _accel(w, 0.8, 0.3, seed=5)
    sim, f = _sim(w, f0, dtype, a)
    sim.kick(0.3)
    out = f.cpu().numpy()
    sim.close()
    g = oracle_grid(w)
    ref = f0
    for ax in (3, 4, 5):
        ref = oracle.sweep(g, ref, ax, 0.3, a)
    assert rel_l1(out, ref) <= (1e-14 if dtype == VP_F64 else 2e-6)


@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
@pytest.mark.parametrize("dtype", [VP_F32, VP_F64])
def test_drift_equals_three_sweeps_and_oracle(bc, dtype):
    w = small_workload(bc, n=(4, 6, 8), nv=(8, 4, 6))
    f0 = structured_f(w.shape, seed=8).astype(NP[dtype]).astype(np.float64)
    a = np.zeros((3,) + w.n)
    tau = 0.11
    sim, f = _sim(w, f0, dtype, a)
    sim.drift(tau)
    out = f.cpu().numpy()
    sim.close()
    sim, f = _sim(w, f0, dtype, a)
    for ax in (2, 1, 0):
        sim.sweep(ax, tau)
    split = f.cpu().numpy()
    sim.close()
    assert np.array_equal(out, split)
    g = oracle_grid(w)
    ref = f0
    for ax in (2, 1, 0):
        ref = oracle.sweep(g, ref, ax, tau)
    assert rel_l1(out, ref) <= (1e-14 if dtype == VP_F64 else 2e-6)
