"""The density of a step's Poisson solve comes from the x sweep's per-workgroup
sums when the grid allows it (256 velocity cells per workgroup, and the
workgroup's tile of new values within 68 KiB of LDS: x lines of up to 64
cells in FP32, 32 in FP64). A step through the C ABI must then agree with the
same step assembled from vp_kick, vp_drift, vp_accel (density from a separate
pass over f) up to the summation order of rho, and with the oracle."""
import numpy as np
import pytest

import oracle
from helpers import oracle_grid, rel_l1, structured_f
from paper_1206_6152_amd import VP_BC_ISOLATED, VP_BC_PERIODIC, VP_F32, VP_F64, Simulator, config_of, inputs

pytestmark = pytest.mark.gpu

NP = {VP_F64: np.float64, VP_F32: np.float32}


def _workload(nx, bc, nv=(8, 8, 4)):
    return inputs.Workload(name="s", n=(nx, 2, 3), nv=nv, L=(0.25 * nx, 0.5, 0.75), vmin=(-1.0, -2.0, -1.5),
                           vmax=(1.5, 2.0, 1.5), G=2.0, bc=bc)


@pytest.mark.parametrize("dtype,nx", [(VP_F32, 3), (VP_F32, 4), (VP_F32, 8), (VP_F32, 12), (VP_F32, 16),
                                      (VP_F32, 24), (VP_F32, 32), (VP_F32, 48), (VP_F32, 64), (VP_F32, 96),
                                      (VP_F64, 4), (VP_F64, 6), (VP_F64, 16), (VP_F64, 24), (VP_F64, 32),
                                      (VP_F64, 48), (VP_F64, 64)])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
def test_step_density_from_x_sweep_sums(dtype, nx, bc):
    import torch
    print("case", dtype, nx, bc, flush=True)
    w = _workload(nx, bc)
    rng = np.random.default_rng(nx)
    f0 = (structured_f(w.shape, seed=nx) + 1e-3 * rng.uniform(0, 1, w.shape)).astype(NP[dtype]).astype(np.float64)
    dt = 0.07
    outs = []
    for mode in ("step", "parts"):
        f = torch.from_numpy(np.ascontiguousarray(f0.astype(NP[dtype]))).to("cuda:0")
        sim = Simulator(config_of(w, dtype), f)
        if mode == "step":
            sim.step(dt)
        else:
            sim.kick(0.5 * dt)
            sim.drift(dt)
            sim.accel()
            sim.kick(0.5 * dt)
        outs.append((f.cpu().numpy().astype(np.float64), sim.get_accel().cpu().numpy()))
        sim.close()
    (fa, aa), (fb, ab) = outs
    scale = np.abs(ab).max()
    assert np.abs(aa - ab).max() <= 1e-12 * scale
    assert rel_l1(fa, fb) <= (1e-14 if dtype == VP_F64 else 1e-6)
    run = oracle.Run(oracle_grid(w), f0)
    run.step(dt)
    assert rel_l1(fa, run.f) <= (1e-13 if dtype == VP_F64 else 2e-6)


@pytest.mark.parametrize("dtype,nx", [(VP_F32, 32), (VP_F64, 32), (VP_F32, 4)])
def test_step_density_from_strided_chunk_groups(dtype, nx):
    # 32^3 velocity cells: 128 chunks of 256 per spatial column. With nx = 32
    # there are 8 chunk groups, each lane adding 16 chunks (the grouping of the
    # benchmark workloads); nx = 4 gives 64 groups of 2 chunks.
    import torch
    print("case", dtype, nx, flush=True)
    w = inputs.Workload(name="s", n=(nx, 2, 2), nv=(32, 32, 32), L=(0.25 * nx, 0.5, 0.5), vmin=(-1.0, -2.0, -1.5),
                        vmax=(1.5, 2.0, 1.5), G=2.0, bc=VP_BC_PERIODIC)
    rng = np.random.default_rng(100 + nx)
    f0 = (structured_f(w.shape, seed=nx) + 1e-3 * rng.uniform(0, 1, w.shape)).astype(NP[dtype]).astype(np.float64)
    dt = 0.05
    outs = []
    for mode in ("step", "parts"):
        f = torch.from_numpy(np.ascontiguousarray(f0.astype(NP[dtype]))).to("cuda:0")
        sim = Simulator(config_of(w, dtype), f)
        if mode == "step":
            sim.step(dt)
        else:
            sim.kick(0.5 * dt)
            sim.drift(dt)
            sim.accel()
            sim.kick(0.5 * dt)
        outs.append((f.cpu().numpy().astype(np.float64), sim.get_accel().cpu().numpy()))
        sim.close()
    (fa, aa), (fb, ab) = outs
    assert np.abs(aa - ab).max() <= 1e-12 * np.abs(ab).max()
    assert rel_l1(fa, fb) <= (1e-14 if dtype == VP_F64 else 1e-6)
    g = oracle_grid(w)
    run = oracle.Run(g, f0)
    run.step(dt)
    # the acceleration the step left behind comes from the x-sweep sums; the
    # oracle's comes from its own density of the drifted f
    np.testing.assert_allclose(aa, run.a, rtol=0, atol=(1e-12 if dtype == VP_F64 else 2e-6) * np.abs(run.a).max())
    assert rel_l1(fa, run.f) <= (1e-13 if dtype == VP_F64 else 2e-6)


@pytest.mark.parametrize("dtype", [VP_F32, VP_F64])
def test_run_with_x_sweep_sums_matches_oracle(dtype):
    # several steps of the fused path (kick pairs, one-pass drift, x sweep sums)
    import torch
    s = inputs.jeans_sigma(0.5, 2 * np.pi)
    w = inputs.Workload(name="r", n=(8, 16, 16), nv=(8, 8, 8), L=(0.5, 1.0, 1.0), vmin=(-4 * s,) * 3,
                        vmax=(4 * s,) * 3, G=1.0, bc=VP_BC_PERIODIC, dt=0.02, steps=3, params=dict(sigma=s, amp=0.05))
    f0 = inputs.initial_f(w)
    f0 *= 1 + 0.05 * np.random.default_rng(3).standard_normal(w.n).reshape(w.n + (1, 1, 1))
    f0 = f0.astype(NP[dtype]).astype(np.float64)
    f = torch.from_numpy(np.ascontiguousarray(f0.astype(NP[dtype]))).to("cuda:0")
    sim = Simulator(config_of(w, dtype), f)
    sim.run(w.steps, w.dt)
    out = f.cpu().numpy().astype(np.float64)
    sim.close()
    run = oracle.Run(oracle_grid(w), f0)
    for _ in range(w.steps):
        run.step(w.dt)
    assert rel_l1(out, run.f) <= (1e-13 if dtype == VP_F64 else 5e-6)
