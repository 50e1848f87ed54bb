"""GPU parity of single directional sweeps T_l(tau) (Sec. 2.1) against the
oracle, through the C ABI: every axis, both boundary types, FP64 and FP32
storage, Courant numbers of both signs below and above one, integer shifts
(bitwise), and line counts that leave a ragged last workgroup."""
import numpy as np
import pytest

import oracle
from helpers import oracle_grid, rel_l1, small_workload, structured_f
from paper_1206_6152_amd import (VP_BC_ISOLATED, VP_BC_PERIODIC, VP_F32, VP_F64, Simulator,
                                 config_of, inputs)

pytestmark = pytest.mark.gpu

NP = {VP_F64: np.float64, VP_F32: np.float32}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def gpu_sweep(w, f0, dtype, axis, tau, accel):
    torch = _torch()
    f = torch.from_numpy(np.ascontiguousarray(f0.astype(NP[dtype]))).to("cuda:0")
    sim = Simulator(config_of(w, dtype), f)
    if accel is not None:
        sim.set_accel(torch.from_numpy(np.ascontiguousarray(accel)))
    sim.sweep(axis, tau)
    out = f.cpu().numpy().astype(np.float64)
    sim.close()
    return out


def random_accel(w, nu_max, tau, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, (3,) + tuple(w.n))
    for l in range(3):
        a[l] *= nu_max * w.dv(l) / abs(tau)
    return a


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
@pytest.mark.parametrize("axis", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("nu_max", [0.9, 2.6])
def test_sweep_matches_oracle(axis, bc, dtype, nu_max):
    print("case", axis, bc, dtype, nu_max, flush=True)
    w = small_workload(bc)
    f0 = structured_f(w.shape, seed=100 + axis)
    f0 = f0.astype(NP[dtype]).astype(np.float64)   # identical inputs on both sides
    g = oracle_grid(w)
    if axis < 3:
        vmax = max(abs(w.vmin[axis]), abs(w.vmax[axis]))
        tau = -nu_max * w.dx(axis) / vmax
        accel = None
    else:
        tau = 0.37
        accel = random_accel(w, nu_max, tau, seed=7 + axis)
    ref = oracle.sweep(g, f0, axis, tau, accel if accel is not None else np.zeros((3,) + w.n))
    out = gpu_sweep(w, f0, dtype, axis, tau, accel)
    scale = np.abs(f0).max()
    if dtype == VP_F64:
        assert np.abs(out - ref).max() <= 1e-13 * scale
        assert rel_l1(out, ref) <= 1e-14
    else:
        assert np.abs(out - ref).max() <= 2e-6 * scale
        assert rel_l1(out, ref) <= 1e-6
    assert out.min() >= -1e-6 * scale   # positivity survives rounding


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_integer_courant_numbers_translate_exactly(axis, dtype):
    # symmetric velocity grid: v_j = (j + 1/2 - N/2) dv, tau = 2 dx / dv gives
    # odd integer shifts; the result is the input moved cell by cell, bitwise
    n = (8, 4, 6)
    nv = (8, 4, 6)
    w = inputs.Workload(name="shift", n=n, nv=nv, L=(2.0, 1.0, 1.5), vmin=(-1.0, -0.5, -0.75),
                        vmax=(1.0, 0.5, 0.75), G=0.0, bc=VP_BC_PERIODIC)
    f0 = structured_f(w.shape, seed=3).astype(NP[dtype]).astype(np.float64)
    tau = 2 * w.dx(axis) / w.dv(axis)
    out = gpu_sweep(w, f0, dtype, axis, tau, None)
    v = w.vc(axis)
    shift = np.rint(v * tau / w.dx(axis)).astype(int)
    ref = np.empty_like(f0)
    for j, s in enumerate(shift):
        src = np.take(f0, [j], axis=axis + 3)
        ref_j = np.roll(src, s, axis=axis)
        idx = [slice(None)] * 6
        idx[axis + 3] = slice(j, j + 1)
        ref[tuple(idx)] = ref_j
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
def test_velocity_integer_shift_outflow(dtype):
    # dv_z = 1/8 and tau = 1/2: a = k/4 gives Courant number k exactly
    w = small_workload(VP_BC_PERIODIC, n=(2, 3, 4), nv=(8, 6, 8))
    f0 = structured_f(w.shape, seed=9).astype(NP[dtype]).astype(np.float64)
    tau = 0.5
    a = np.zeros((3,) + w.n)
    a[2] = (np.arange(np.prod(w.n)).reshape(w.n) % 5 - 2) * 0.25   # shifts -2..2
    out = gpu_sweep(w, f0, dtype, 5, tau, a)
    ref = oracle.sweep(oracle_grid(w), f0, 5, tau, a)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
def test_ragged_line_counts(dtype):
    # 3*6*12 spatial x 2*3*4 velocity: no axis gives a whole number of workgroups
    w = small_workload(VP_BC_PERIODIC, n=(3, 6, 12), nv=(2, 3, 4))
    f0 = structured_f(w.shape, seed=21).astype(NP[dtype]).astype(np.float64)
    g = oracle_grid(w)
    for axis in range(6):
        tau = 0.21 if axis >= 3 else 0.05
        accel = random_accel(w, 0.8, tau, seed=axis)
        ref = oracle.sweep(g, f0, axis, tau, accel)
        out = gpu_sweep(w, f0, dtype, axis, tau, accel if axis >= 3 else None)
        tol = 1e-14 if dtype == VP_F64 else 1e-6
        assert rel_l1(out, ref) <= tol, axis


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
@pytest.mark.parametrize("nvl", [8, 24, 32, 48, 64])
def test_velocity_line_lengths_of_the_workloads(nvl, dtype):
    # the velocity line lengths of the benchmark workloads, on every velocity
    # axis, with enough lines for several full workgroups and a ragged tail
    w = small_workload(VP_BC_PERIODIC, n=(2, 3, 2), nv=(nvl, 3, nvl))
    f0 = structured_f(w.shape, seed=nvl).astype(NP[dtype]).astype(np.float64)
    g = oracle_grid(w)
    for axis in (3, 4, 5):
        tau = 0.3
        accel = random_accel(w, 0.95, tau, seed=axis + nvl)
        ref = oracle.sweep(g, f0, axis, tau, accel)
        out = gpu_sweep(w, f0, dtype, axis, tau, accel)
        tol = 1e-14 if dtype == VP_F64 else 1e-6
        assert rel_l1(out, ref) <= tol, axis


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
@pytest.mark.parametrize("nl", [24, 32, 48, 64, 96, 128])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
def test_position_line_lengths_of_the_workloads(nl, bc, dtype):
    # position lines of the workloads' lengths along z (mixed-sign waves), y
    # and x, periodic and outflow
    w = small_workload(bc, n=(nl, 2, nl), nv=(2, 3, 4))
    w = inputs.Workload(name="pos", n=w.n, nv=w.nv, L=tuple(0.25 * x for x in w.n), vmin=(-1.0, -2.0, -1.5),
                        vmax=(1.5, 2.0, 1.5), G=1.0, bc=bc)
    f0 = structured_f(w.shape, seed=nl + bc).astype(NP[dtype]).astype(np.float64)
    g = oracle_grid(w)
    for axis in (2, 0):
        vmax = max(abs(w.vmin[axis]), abs(w.vmax[axis]))
        tau = 0.8 * w.dx(axis) / vmax
        ref = oracle.sweep(g, f0, axis, tau, np.zeros((3,) + w.n))
        out = gpu_sweep(w, f0, dtype, axis, tau, None)
        err = np.abs(out - ref).max() / np.abs(f0).max()
        if err > (1e-13 if dtype == VP_F64 else 3e-6):
            bad = np.argwhere(np.abs(out - ref) > (1e-13 if dtype == VP_F64 else 3e-6) * np.abs(f0).max())
            print("axis", axis, "max err", err, "bad count", len(bad), "first", bad[:8].tolist(), flush=True)
        tol = 1e-14 if dtype == VP_F64 else 1e-6
        assert rel_l1(out, ref) <= tol, (axis, rel_l1(out, ref))
