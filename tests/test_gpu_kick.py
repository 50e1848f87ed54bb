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


CASES = [(VP_F32, 8), (VP_F32, 16), (VP_F32, 24), (VP_F32, 32), (VP_F32, 48), (VP_F32, 64),
         (VP_F64, 8), (VP_F64, 16), (VP_F64, 24), (VP_F64, 32), (VP_F64, 48), (VP_F64, 64)]


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


@pytest.mark.parametrize("dtype,nv", [(VP_F32, 32), (VP_F64, 24), (VP_F64, 32), (VP_F32, 48), (VP_F64, 48)])
@pytest.mark.parametrize("reps", [1, 2])
def test_kick_degenerate_accelerations(dtype, nv, reps):
    # spatial cells with no acceleration (nu = 0 on every axis), with nu at or
    # next to a whole number of cells (alpha near 0), with |nu| beyond the
    # block (everything leaves through the outflow boundary), and mixes of
    # these over the three axes; one or two vp_kick calls must equal the
    # single sweeps bit for bit
    print("case", dtype, nv, reps, flush=True)
    w = small_workload(VP_BC_PERIODIC, n=(2, 2, 2), nv=(nv, nv, nv))
    f0 = structured_f(w.shape, seed=nv + 3).astype(NP[dtype]).astype(np.float64)
    tau = 0.5
    dv = np.array([w.dv(l) for l in range(3)])
    nus = np.array([[0.0, 0.0, 0.0], [1.0, -2.0, 3.0], [nv + 5.5, -(nv + 0.25), 2.0 * nv],
                    [0.0, -(nv + 1.0), 0.6], [-1.3, 0.0, 0.0], [0.25, 0.5, -0.75], [-7.0, 7.5, -0.0],
                    [nv - 1.0, -(nv - 0.5), nv]])
    a = np.zeros((3,) + w.n)
    for c in range(8):
        ix, iy, iz = c >> 2, (c >> 1) & 1, c & 1
        a[:, ix, iy, iz] = nus[c] * dv / tau
    outs = []
    for mode in ("kick", "split"):
        sim, f = _sim(w, f0, dtype, a)
        for _ in range(reps):
            if mode == "kick":
                sim.kick(tau)
            else:
                for ax in (3, 4, 5):
                    sim.sweep(ax, tau)
        outs.append(f.cpu().numpy())
        sim.close()
    assert np.array_equal(outs[0], outs[1])
    g = oracle_grid(w)
    ref = f0
    for _ in range(reps):
        for ax in (3, 4, 5):
            ref = oracle.sweep(g, ref, ax, tau, a)
    assert rel_l1(outs[0], ref) <= (1e-14 if dtype == VP_F64 else 2e-6)
    # cells whose nu passes the block on some axis are empty afterwards
    assert not outs[0][0, 1, 0].any()


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


@pytest.mark.parametrize("dtype", [VP_F32, VP_F64])
@pytest.mark.parametrize("plane", [16, 24, 32, 48, 64])
@pytest.mark.parametrize("nu_max", [0.7, 2.4])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
def test_one_pass_drift_planes(plane, dtype, nu_max, bc):
    # square (y, z) planes take the one-pass T_y T_z; it must equal the single
    # sweeps bit for bit and the oracle within tolerance
    print("case", plane, dtype, nu_max, bc, flush=True)
    w = small_workload(bc, n=(2, plane, plane), nv=(4, 4, 8))
    w = w.__class__(name="d", n=w.n, nv=w.nv, L=tuple(0.25 * x for x in w.n), vmin=(-1.0, -2.0, -1.5),
                    vmax=(1.5, 2.0, 1.5), G=1.0, bc=bc)
    rng = np.random.default_rng(plane)
    f0 = (structured_f(w.shape, seed=plane) + 1e-3 * rng.uniform(0, 1, w.shape)).astype(NP[dtype]).astype(np.float64)
    a = np.zeros((3,) + w.n)
    tau = nu_max * 0.25 / 2.0
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


@pytest.mark.parametrize("dtype", [VP_F32, VP_F64])
@pytest.mark.parametrize("shape", [((4, 16, 16), (16, 16, 16)), ((2, 6, 4), (8, 8, 8)), ((2, 3, 4), (8, 12, 16)),
                                   ((2, 2, 4), (32, 32, 32)), ((2, 2, 2), (48, 48, 48)),
                                   ((2, 2, 2), (64, 64, 64)), ((1, 2, 3), (48, 48, 48))])
def test_run_equals_repeated_steps(shape, dtype):
    # vp_run merges the closing and opening half kicks of consecutive steps;
    # the result must be the same bits as separate vp_step calls
    n, nv = shape
    from paper_1206_6152_amd import inputs
    s = inputs.jeans_sigma(0.5, 2 * np.pi)
    w = inputs.Workload(name="r", n=n, nv=nv, L=tuple(x / 16.0 for x in n), vmin=(-4 * s,) * 3, vmax=(4 * s,) * 3,
                        G=1.0, bc=VP_BC_PERIODIC, dt=0.02, steps=4, params=dict(sigma=s, amp=0.05))
    f0 = inputs.initial_f(w)
    f0 *= 1 + 0.05 * np.random.default_rng(1).standard_normal(w.n).reshape(w.n + (1, 1, 1))
    import torch
    outs = []
    for mode in ("run", "step"):
        f = torch.from_numpy(np.ascontiguousarray(f0.astype(NP[dtype]))).to("cuda:0")
        sim = Simulator(config_of(w, dtype), f)
        if mode == "run":
            sim.run(w.steps, w.dt)
        else:
            for _ in range(w.steps):
                sim.step(w.dt)
        outs.append((f.cpu().numpy(), sim.get_accel().cpu().numpy()))
        sim.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("dtype,plane,nx,nv", [(VP_F32, 16, 48, (8, 8, 16)), (VP_F32, 24, 32, (8, 8, 16)),
                                                (VP_F32, 32, 12, (8, 8, 16)), (VP_F32, 32, 3, (2, 3, 16)),
                                                (VP_F32, 16, 1, (1, 3, 64)), (VP_F64, 32, 3, (1, 3, 16)),
                                                (VP_F64, 24, 1, (1, 3, 16)), (VP_F64, 16, 3, (1, 3, 32)),
                                                (VP_F32, 48, 8, (4, 4, 8)), (VP_F32, 64, 8, (2, 4, 16)),
                                                (VP_F64, 48, 2, (4, 4, 8)), (VP_F64, 64, 2, (2, 4, 16))])
def test_one_pass_drift_many_tiles_per_workgroup(dtype, plane, nx, nv):
    # a workgroup walks several (x, velocity chunk) tiles (four, or two for
    # FP64 planes of 16, 24 and 48); the tile counts here include ragged ends
    # (9 and 3 tiles in FP32; 9, 3 and 9 in FP64). The FP64 48-planes take
    # chunks narrower than a cache line, and their case has a multiple of 8
    # workgroup units, so the workgroups that share lines are grouped per XCD.
    # FP32 planes of 32, 48 and 64 and FP64 planes of 32 hold two lines per
    # lane; FP64 64-planes keep two plain sweeps.
    print("case", dtype, plane, nx, nv, flush=True)
    w = small_workload(VP_BC_PERIODIC, n=(nx, plane, plane), nv=nv)
    w = w.__class__(name="d", n=w.n, nv=w.nv, L=tuple(0.25 * x for x in w.n), vmin=(-1.0, -2.0, -1.5),
                    vmax=(1.5, 2.0, 1.5), G=1.0, bc=VP_BC_PERIODIC)
    rng = np.random.default_rng(plane + nx)
    f0 = (structured_f(w.shape, seed=plane) + 1e-3 * rng.uniform(0, 1, w.shape)).astype(NP[dtype]).astype(np.float64)
    a = np.zeros((3,) + w.n)
    tau = 1.3 * 0.25 / 2.0
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


@pytest.mark.parametrize("dtype,plane,nv", [(VP_F32, 32, (2, 8, 6)), (VP_F32, 48, (2, 8, 6)), (VP_F32, 64, (1, 64, 6)),
                                            (VP_F32, 64, (2, 4, 6)), (VP_F64, 32, (2, 4, 6)),
                                            (VP_F32, 32, (2, 16, 3)), (VP_F32, 64, (1, 16, 3))])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
def test_one_pass_drift_pairs_of_cells(dtype, plane, nv, bc):
    # the two-lines-per-lane drift holds velocity cells 2p and 2p + 1 in one
    # lane: with nv_z = 6 the pair (2, 3) straddles vz = 0, so its two z lines
    # run in opposite orientations while sharing the y sweep. The 64-planes
    # take half-line chunks whose two workgroups per line are grouped per XCD
    # (24 chunks); with 3 chunks they cannot pair up and the drift takes the
    # single sweeps, as it does with nv_z odd, where a pair would straddle a
    # vz row.
    print("case", dtype, plane, nv, bc, flush=True)
    w = small_workload(bc, n=(3, plane, plane), nv=nv)
    w = w.__class__(name="d", n=w.n, nv=w.nv, L=tuple(0.25 * x for x in w.n), vmin=(-1.0, -2.0, -1.5),
                    vmax=(1.5, 2.0, 1.5), G=1.0, bc=bc)
    rng = np.random.default_rng(plane + nv[2])
    f0 = (structured_f(w.shape, seed=plane) + 1e-3 * rng.uniform(0, 1, w.shape)).astype(NP[dtype]).astype(np.float64)
    a = np.zeros((3,) + w.n)
    tau = 1.7 * 0.25 / 2.0
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
