"""GPU parity of the reverse mode through the C ABI against the oracle's reverse
mode (single sweeps with their acceleration adjoints, the transposed gravity
map, short multi-step gradients), and of the adjoint workload (16^3 x 24^3,
40 steps, checkpoints every 8) against central finite differences of the GPU
forward map in FP64 and against the FP64 gradient for the FP32 path."""
import numpy as np
import pytest

import oracle
from helpers import oracle_grid, rel_l1, small_workload, structured_f
from paper_1206_6152_amd import VP_BC_ISOLATED, VP_BC_PERIODIC, VP_F32, VP_F64, Simulator, config_of, inputs

pytestmark = pytest.mark.gpu

NP = {VP_F64: np.float64, VP_F32: np.float32}


def _t():
    import torch
    assert torch.cuda.is_available()
    return torch


def _dev(x, dtype=None):
    torch = _t()
    return torch.from_numpy(np.ascontiguousarray(x if dtype is None else x.astype(dtype))).to("cuda:0")


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
@pytest.mark.parametrize("axis", [0, 1, 2, 3, 4, 5])
def test_sweep_adjoint_matches_oracle(axis, bc, dtype):
    print("case", axis, bc, dtype, flush=True)
    w = small_workload(bc, n=(4, 6, 8), nv=(12, 8, 6))
    rng = np.random.default_rng(40 + axis)
    f_in = (structured_f(w.shape, 50 + axis) + 0.01 + 1e-3 * rng.uniform(0, 1, w.shape))
    f_in = f_in.astype(NP[dtype]).astype(np.float64)
    lam = rng.standard_normal(w.shape).astype(NP[dtype]).astype(np.float64)
    tau = 0.31 if axis >= 3 else -0.9 * w.dx(axis) / max(abs(w.vmin[axis]), abs(w.vmax[axis]))
    a = rng.uniform(-1, 1, (3,) + w.n) * 1.3 * np.array([w.dv(l) for l in range(3)]).reshape(3, 1, 1, 1) / abs(tau)
    g = oracle_grid(w)
    ref_lam, ref_la = oracle.sweep_vjp(g, f_in, axis, tau, lam, a)
    torch = _t()
    f = _dev(f_in, NP[dtype])
    sim = Simulator(config_of(w, dtype), f)
    sim.set_accel(_dev(a))
    lam_d = _dev(lam, NP[dtype])
    la_d = torch.zeros((3,) + w.n, dtype=torch.float64, device="cuda:0")
    sim.sweep_adjoint(axis, tau, _dev(f_in, NP[dtype]), lam_d, la_d)
    out = lam_d.cpu().numpy().astype(np.float64)
    la = la_d.cpu().numpy()
    sim.close()
    tol = 1e-12 if dtype == VP_F64 else 2e-5
    assert rel_l1(out, ref_lam) <= tol
    if axis >= 3:
        assert rel_l1(la, ref_la) <= (1e-11 if dtype == VP_F64 else 1e-4)


@pytest.mark.parametrize("dtype,nv", [(VP_F32, 8), (VP_F32, 16), (VP_F32, 24), (VP_F64, 8)])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
def test_one_pass_reverse_kick_equals_three_reverse_sweeps(dtype, nv, bc):
    # vp_kick_adjoint rebuilds T_vx x and T_vy T_vx x on chip and runs the
    # three reverse line updates there: lam and the acceleration adjoint must
    # be the bits of vp_sweep_adjoint along vz, vy and vx at those states.
    # Accelerations of both signs, with whole-cell shifts (|nu| up to 2.3).
    print("case", dtype, nv, bc, flush=True)
    torch = _t()
    w = small_workload(bc, n=(2, 3, 2), nv=(nv, nv, nv))
    rng = np.random.default_rng(nv + 7 * bc)
    x = (structured_f(w.shape, 60 + nv) + 0.01 + 1e-3 * rng.uniform(0, 1, w.shape)).astype(NP[dtype])
    lam0 = rng.standard_normal(w.shape).astype(NP[dtype])
    tau = 0.27
    a = rng.uniform(-1, 1, (3,) + w.n) * 2.3 * np.array([w.dv(l) for l in range(3)]).reshape(3, 1, 1, 1) / tau
    g = _dev(x)
    sim = Simulator(config_of(w, dtype), g)
    sim.set_accel(_dev(a))
    sim.sweep(3, tau)
    in1 = g.clone()
    sim.sweep(4, tau)
    in2 = g.clone()
    lam_s = _dev(lam0)
    la_s = torch.zeros((3,) + w.n, dtype=torch.float64, device="cuda:0")
    sim.sweep_adjoint(5, tau, in2, lam_s, la_s)
    sim.sweep_adjoint(4, tau, in1, lam_s, la_s)
    sim.sweep_adjoint(3, tau, _dev(x), lam_s, la_s)
    lam_f = _dev(lam0)
    la_f = torch.zeros((3,) + w.n, dtype=torch.float64, device="cuda:0")
    sim.kick_adjoint(tau, _dev(x), lam_f, la_f)
    lam_n = _dev(lam0)
    sim.kick_adjoint(tau, _dev(x), lam_n)          # no acceleration adjoint wanted
    sim.close()
    assert torch.equal(lam_f, lam_s)
    assert torch.equal(la_f, la_s)
    assert torch.equal(lam_n, lam_s)
    assert float(la_s.abs().sum()) > 0


def test_reverse_kick_unsupported_grid():
    from paper_1206_6152_amd import VPError, _lib
    torch = _t()
    w = small_workload(VP_BC_PERIODIC, n=(2, 2, 2), nv=(32, 32, 32))
    x = _dev(np.full(w.shape, 0.5, dtype=np.float32))
    sim = Simulator(config_of(w, VP_F32), x)
    with pytest.raises(VPError) as e:
        sim.kick_adjoint(0.1, x, x.clone())
    sim.close()
    assert e.value.code == _lib.VP_EUNSUPPORTED


@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
def test_accel_adjoint_matches_oracle(bc):
    w = small_workload(bc, n=(4, 6, 8), nv=(4, 3, 2))
    rng = np.random.default_rng(3)
    la = rng.standard_normal((3,) + w.n)
    ref = oracle.accel_vjp(oracle_grid(w), la)
    torch = _t()
    f = _dev(np.ones(w.shape))
    sim = Simulator(config_of(w, VP_F64), f)
    lam = torch.zeros(w.shape, dtype=torch.float64, device="cuda:0")
    sim.accel_adjoint(_dev(la), lam)
    out = lam.cpu().numpy()
    sim.close()
    assert rel_l1(out, ref) <= 1e-12


def _tiny(bc):
    if bc == VP_BC_PERIODIC:
        s = inputs.jeans_sigma(0.5, 2 * np.pi)
        w = inputs.Workload(name="t", n=(4, 2, 2), nv=(8, 4, 4), L=(1.0, 0.5, 0.5), vmin=(-4 * s,) * 3,
                            vmax=(4 * s,) * 3, G=1.0, bc=0, dt=0.04, steps=5, params=dict(sigma=s, amp=0.1))
        f0 = inputs.initial_f(w)
        f0 *= 1 + 0.05 * np.random.default_rng(4).standard_normal(w.n).reshape(w.n + (1, 1, 1))
    else:
        w = inputs.Workload(name="t", n=(4, 4, 4), nv=(6, 6, 6), L=(4.0, 4.0, 4.0), vmin=(-2.0,) * 3,
                            vmax=(2.0,) * 3, G=1.0, bc=1, dt=0.2, steps=3, params=dict(sigma=0.6))
        X = np.meshgrid(*[w.xc(l) for l in range(3)], indexing="ij")
        dens = np.exp(-(X[0] ** 2 + X[1] ** 2 + X[2] ** 2) / 2.0)
        f0 = dens.reshape(w.n + (1, 1, 1)) * inputs.maxwellian(w, 0.6).reshape((1, 1, 1) + w.nv)
    # symmetric data has exactly tied line maxima; rounding of either side then
    # decides which cell receives f_inf's adjoint (both are valid), so break
    # the ties well above rounding
    f0 = f0 * (1 + 1e-4 * np.random.default_rng(11).uniform(0, 1, f0.shape))
    return w, f0


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
@pytest.mark.parametrize("ckpt", [1, 2, 8])
def test_grad_matches_oracle(bc, dtype, ckpt):
    w, f0 = _tiny(bc)
    f0 = f0.astype(NP[dtype]).astype(np.float64)
    L_ref, g_ref = oracle.grad(oracle_grid(w), f0, w.steps, w.dt)
    f = _dev(f0, NP[dtype])
    sim = Simulator(config_of(w, dtype), f)
    L, g = sim.grad(w.steps, w.dt, ckpt)
    out = g.cpu().numpy().astype(np.float64)
    fin = f.cpu().numpy().astype(np.float64)
    sim.close()
    run = oracle.Run(oracle_grid(w), f0)
    for _ in range(w.steps):
        run.step(w.dt)
    print("grad", bc, dtype, ckpt, "L", L, L_ref, "rel L1", rel_l1(out, g_ref), flush=True)
    if dtype == VP_F64:
        assert L == pytest.approx(L_ref, rel=1e-12)
        assert rel_l1(out, g_ref) <= 1e-10
        assert rel_l1(fin, run.f) <= 1e-12      # f ends at the final state
    else:
        assert L == pytest.approx(L_ref, rel=1e-5)
        assert rel_l1(out, g_ref) <= 1e-3
        assert rel_l1(fin, run.f) <= 1e-5


def test_adjoint_workload_against_finite_differences():
    # the 16^3 x 24^3 adjoint workload: Jeans sigma, delta ~ N(0, 1e-3^2) per
    # spatial cell, 40 steps, checkpoints every 8; FD of the GPU FP64 forward
    torch = _t()
    from paper_1206_6152_amd.autograd import field_energy, initial_f
    w = inputs.jeans_adjoint_16_24()
    dens, m = inputs.separable_factors(w)
    delta = _dev(dens - 1.0).requires_grad_(True)
    m_v = _dev(m)
    L64 = field_energy(delta, m_v, w, VP_F64, w.steps, w.dt, 8)
    L64.backward()
    g64 = delta.grad.detach().clone()
    delta.grad = None
    L32 = field_energy(delta, m_v, w, VP_F32, w.steps, w.dt, 8)
    L32.backward()
    g32 = delta.grad.detach().clone()
    r32 = float((g32 - g64).abs().sum() / g64.abs().sum())
    print("L64", float(L64), "L32", float(L32), "FP32 vs FP64 gradient rel L1", r32, flush=True)
    assert r32 <= 1e-3

    def loss_at(d):
        f = initial_f(d, m_v, 1.0, torch.float64)
        sim = Simulator(config_of(w, VP_F64), f)
        sim.run(w.steps, w.dt)
        e = sim.energy()
        sim.close()
        return -e[1]

    # Central differences along 8 random unit directions and 8 single cells,
    # errors relative to FD (and, printed, to |grad| |d|). The limited map is
    # piecewise smooth: a step crosses corrector and line-maximum kinks, where
    # the central difference averages the slopes of neighbouring pieces and the
    # reverse mode takes the piece the state is in. At the stated step
    # eps = 1e-4 most random directions agree to 1e-4; as the step shrinks the
    # kinks crossed thin out and every direction converges to the reverse mode
    # (measured: <= 2.3e-5 at eps = 1e-7, against up to 1.5e-3 at 1e-4 on single
    # cells and 3.9e-4 on the random direction whose derivative cancels to
    # 4e-4 of |grad| |d|).
    rng = np.random.default_rng(6152)
    dirs = []
    for _ in range(8):
        d = rng.standard_normal(w.n)
        dirs.append(d / np.linalg.norm(d))
    cells = [tuple(int(rng.integers(0, n)) for n in w.n) for _ in range(8)]
    for c in cells:
        e = np.zeros(w.n)
        e[c] = 1.0
        dirs.append(e)
    gnorm = float(g64.norm())

    def fd_at(d, h):
        return (loss_at(delta.detach() + h * d) - loss_at(delta.detach() - h * d)) / (2 * h)
    rel4, rel7 = [], []
    for k, d in enumerate(dirs):
        d = _dev(d)
        an = float((g64 * d).sum())
        fd4, fd7 = fd_at(d, 1e-4), fd_at(d, 1e-7)
        rel4.append(abs(an - fd4) / abs(fd4))
        rel7.append(abs(an - fd7) / abs(fd7))
        kind = "random unit" if k < 8 else "cell %s" % (cells[k - 8],)
        print("direction %2d (%s): adjoint %.10e  FD(1e-4) %.10e  |err|/|FD| %.2e  |err|/(|g||d|) %.2e  "
              "FD(1e-7) |err|/|FD| %.2e" % (k, kind, an, fd4, rel4[-1], abs(an - fd4) / (gnorm * float(d.norm())),
                                            rel7[-1]), flush=True)
    rel4 = np.array(rel4)
    print("eps 1e-4: random directions within 1e-4: %d of 8, worst %.2e; single cells worst %.2e; "
          "eps 1e-7: worst %.2e" % (int((rel4[:8] <= 1e-4).sum()), rel4[:8].max(), rel4[8:].max(), max(rel7)),
          flush=True)
    assert (rel4[:8] <= 1e-4).sum() >= 7 and rel4[:8].max() <= 1e-3
    assert rel4[8:].max() <= 5e-3
    assert max(rel7) <= 1e-4


def test_adjoint_workload_grid_gradient_matches_oracle():
    # vp_grad on the adjoint workload's grid (16^3 x 24^3) for one checkpoint
    # segment (8 steps) against the oracle's FP64 reverse mode, which keeps every
    # state of the forward run: FP64 with checkpoints every 8 and every 3 steps,
    # and the FP32-stored path
    import threading
    torch = _t()
    w = inputs.jeans_adjoint_16_24()
    steps = 8
    f0 = inputs.initial_f(w).astype(np.float32).astype(np.float64)
    g = oracle_grid(w)
    box = {}
    th = threading.Thread(target=lambda: box.update(ref=oracle.grad(g, f0, steps, w.dt)), daemon=True)
    th.start()
    out = {}
    for dtype, ckpt in ((VP_F64, 8), (VP_F64, 3), (VP_F32, 8)):
        f = _dev(f0, NP[dtype])
        sim = Simulator(config_of(w, dtype), f)
        L, gr = sim.grad(steps, w.dt, ckpt)
        out[(dtype, ckpt)] = (L, gr.cpu().numpy().astype(np.float64))
        sim.close()
        del f, gr
    th.join()
    L_ref, g_ref = box["ref"]
    for (dtype, ckpt), (L, gr) in out.items():
        err = rel_l1(gr, g_ref)
        print("%s ckpt %d: L %.12e vs %.12e, gradient rel L1 %.2e" % (
            "FP64" if dtype == VP_F64 else "FP32", ckpt, L, L_ref, err), flush=True)
        if dtype == VP_F64:
            assert L == pytest.approx(L_ref, rel=1e-11)
            assert err <= 1e-10
        else:
            assert L == pytest.approx(L_ref, rel=1e-3)
            assert err <= 2e-3


def test_grad_fp64_register_kick_blocks_match_oracle():
    # FP64 32^3 velocity blocks take the one-pass kick that holds the block in
    # registers, also where a segment's recomputed first half kick is written
    # straight into the next state's buffer; the gradient must match the
    # oracle's and be the same bits for every checkpoint interval
    s = inputs.jeans_sigma(0.5, 2 * np.pi)
    w = inputs.Workload(name="t", n=(2, 2, 2), nv=(32, 32, 32), L=(0.5, 0.5, 0.5), vmin=(-4 * s,) * 3,
                        vmax=(4 * s,) * 3, G=1.0, bc=0, dt=0.04, steps=3, params=dict(sigma=s, amp=0.1))
    f0 = inputs.initial_f(w)
    f0 *= 1 + 0.05 * np.random.default_rng(5).standard_normal(w.n).reshape(w.n + (1, 1, 1))
    f0 = f0 * (1 + 1e-4 * np.random.default_rng(12).uniform(0, 1, f0.shape))
    L_ref, g_ref = oracle.grad(oracle_grid(w), f0, w.steps, w.dt)
    outs = []
    for ckpt in (1, 2, 8):
        f = _dev(f0, np.float64)
        sim = Simulator(config_of(w, VP_F64), f)
        sim.profile(True)
        L, g = sim.grad(w.steps, w.dt, ckpt)
        phases = sim.profile_read()
        outs.append((L, g.cpu().numpy(), f.cpu().numpy()))
        sim.close()
        assert phases["kick"][1] + phases["kick2"][1] > 0 and phases["vz"][1] == 0
    print("grad FP64 32^3 blocks: L", outs[0][0], L_ref, "rel L1", rel_l1(outs[0][1], g_ref), flush=True)
    assert outs[0][0] == pytest.approx(L_ref, rel=1e-12)
    assert rel_l1(outs[0][1], g_ref) <= 1e-10
    for L, g, fin in outs[1:]:
        assert L == outs[0][0]
        assert np.array_equal(g, outs[0][1])
        assert np.array_equal(fin, outs[0][2])


@pytest.mark.parametrize("dtype", [VP_F64, VP_F32])
@pytest.mark.parametrize("bc", [VP_BC_PERIODIC, VP_BC_ISOLATED])
def test_grad_same_bits_for_every_checkpoint_interval(bc, dtype):
    # the states a segment recomputes (first half kick written straight into
    # the next state's buffer where the velocity block fits on chip, a copy and
    # an in-place kick otherwise) are those of the forward run, bit for bit
    w, f0 = _tiny(bc)
    f0 = f0.astype(NP[dtype]).astype(np.float64)
    outs = []
    for ckpt in (1, 2, 3, 8):
        f = _dev(f0, NP[dtype])
        sim = Simulator(config_of(w, dtype), f)
        L, g = sim.grad(w.steps, w.dt, ckpt)
        outs.append((L, g.cpu().numpy(), f.cpu().numpy()))
        sim.close()
    for L, g, fin in outs[1:]:
        assert L == outs[0][0]
        assert np.array_equal(g, outs[0][1])
        assert np.array_equal(fin, outs[0][2])


def test_benchmark_grid_gradient_fp32_against_fp64_and_finite_differences():
    # The reverse mode on the benchmark's grid (32^3 x 32^3, 1.07e9 cells) for 10
    # steps with checkpoints every 5: the call holds ceil(10/5) + 5 + 1 = 8 copies
    # of f (34 GB in FP32, 69 GB in FP64). The FP32 gradient with respect to the
    # initial density contrast is compared with the FP64 one, and both with
    # central differences of the FP64 forward map along the perturbation's own
    # mode and along random unit directions.
    torch = _t()
    from paper_1206_6152_amd.autograd import field_energy, initial_f
    w = inputs.jeans_32_32()
    steps, ckpt = 10, 5
    dens, m = inputs.separable_factors(w)
    delta = _dev(dens - 1.0).requires_grad_(True)
    m_v = _dev(m)
    grads = {}
    for dtype in (VP_F64, VP_F32):
        L = field_energy(delta, m_v, w, dtype, steps, w.dt, ckpt)
        L.backward()
        grads[dtype] = (float(L.detach()), delta.grad.detach().clone())
        delta.grad = None
        torch.cuda.empty_cache()
    (L64, g64), (L32, g32) = grads[VP_F64], grads[VP_F32]
    r32 = float((g32 - g64).abs().sum() / g64.abs().sum())
    print("L64 %.12e L32 %.12e, FP32 vs FP64 gradient rel L1 %.2e" % (L64, L32, r32), flush=True)
    assert L32 == pytest.approx(L64, rel=1e-4)
    assert r32 <= 1e-3

    def loss_at(d):
        f = initial_f(d, m_v, 1.0, torch.float64)
        sim = Simulator(config_of(w, VP_F64), f)
        sim.run(steps, w.dt)
        e = sim.energy()
        sim.close()
        del f
        return -e[1]

    rng = np.random.default_rng(32)
    mode = (dens - 1.0) / np.linalg.norm(dens - 1.0)
    dirs = [("cosine mode", mode)]
    for i in range(3):
        d = rng.standard_normal(w.n)
        dirs.append(("random unit %d" % i, d / np.linalg.norm(d)))
    eps = 1e-4
    for name, d in dirs:
        d = _dev(d)
        fd = (loss_at(delta.detach() + eps * d) - loss_at(delta.detach() - eps * d)) / (2 * eps)
        a64, a32 = float((g64 * d).sum()), float((g32 * d).sum())
        print("%s: FD %.10e  FP64 adjoint %.10e (%.2e)  FP32 adjoint %.10e (%.2e)" % (
            name, fd, a64, abs(a64 - fd) / abs(fd), a32, abs(a32 - fd) / abs(fd)), flush=True)
        assert abs(a64 - fd) <= 1e-4 * abs(fd)
        assert abs(a32 - fd) <= 1e-3 * abs(fd)
