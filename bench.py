#!/usr/bin/env python3
"""Throughput of the six-dimensional PFC Vlasov-Poisson step on one MI355X.

Workload (default): the Jeans-instability cube, periodic unit box, k/k_J = 0.5,
A = 0.01 cosine along x on a Maxwellian, 32^3 spatial x 32^3 velocity cells
(1.07e9 phase-space cells), fixed dt (CFL 0.5). One step is one application of
the split operator product (nine directional sweeps, one density moment and
one Poisson solve). Inputs are synthetic and built on the device before the
timed region; f stays resident in HBM.

Prints ONE JSON line: value = phase-space cell updates per second with f stored
and swept in FP32 (density/Poisson/acceleration in FP64), plus the FP64-stored
rate, the roofline of the dominant sweep kernel (HIP events around every
launch on the library's stream), per-phase times in the layout of the paper's
Table 1, the measured device-copy bandwidth, and the CPU oracle's rate on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0   # MI355X HBM3E, AMD public specification
# Vector ALU issue rate without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane-operations/s (= 157.3 TFLOP/s FP32 / 2 for FMA / 2 for packed pairs).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Arithmetic of one cell in one sweep: line maximum (a max3 covers two cells: 0.5),
# f_{k+1} - f_k (1), 2 f_k (1), 2 f_inf - 2 f_k (1), two clamps (2),
# q_k = fma(c2, Lm, fma(c1, Lp, f_k)) (2), q_{k-1} - q_k (1), g_k = fma(alpha, q_{k-1} - q_k, f_k) (1).
OPS_PER_CELL_SWEEP = 9.5
METRIC = "phase-space cell updates/s (FP32 vs FP64 GPU) + % HBM roofline"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_f(w, torch_dtype, device):
    """f = (spatial factor) x (velocity factor), or the King distribution
    rho1 (2 pi)^(-3/2) (exp(E) - 1) for E = Psi(x) - v^2/2 > 0 (isolated
    workloads), formed on the device in FP64 and rounded once to the storage
    type, chunk by chunk."""
    import numpy as np
    import torch
    from paper_1206_6152_amd import inputs
    if w.bc == 1:
        psi = torch.from_numpy(inputs.king_psi(w).reshape(-1)).to(device)
        V = np.meshgrid(*[w.vc(l) for l in range(3)], indexing="ij")
        hv2 = torch.from_numpy((0.5 * (V[0] ** 2 + V[1] ** 2 + V[2] ** 2)).reshape(-1)).to(device)
        pref = inputs.king_prefactor(w.params["W0"])
        f = torch.empty(w.shape, dtype=torch_dtype, device=device)
        fv = f.view(psi.numel(), hv2.numel())
        chunk = max(1, (1 << 27) // hv2.numel())
        for i in range(0, psi.numel(), chunk):
            e = psi[i:i + chunk, None] - hv2[None, :]
            fv[i:i + chunk] = torch.where(e > 0, pref * torch.expm1(e.clamp(min=0)), torch.zeros_like(e)).to(torch_dtype)
        torch.cuda.synchronize()
        return f
    dens, m = inputs.separable_factors(w)
    d = torch.from_numpy(dens.reshape(-1)).to(device)
    mv = torch.from_numpy(m.reshape(-1)).to(device)
    np_, nv3 = d.numel(), mv.numel()
    f = torch.empty(w.shape, dtype=torch_dtype, device=device)
    fv = f.view(np_, nv3)
    chunk = max(1, (1 << 27) // nv3)
    for i in range(0, np_, chunk):
        fv[i:i + chunk] = (d[i:i + chunk, None] * mv[None, :]).to(torch_dtype)
    torch.cuda.synchronize()
    return f


def copy_bandwidth(f):
    """GB/s (read + write) of the library's plain 16-byte-per-lane copy of a
    buffer of f's size: the practical HBM ceiling the passes are compared with."""
    import torch
    from paper_1206_6152_amd._lib import vp_stream_copy
    g = torch.empty_like(f)
    stream = torch.cuda.current_stream().cuda_stream
    nb = f.numel() * f.element_size()
    vp_stream_copy(f.data_ptr(), g.data_ptr(), nb, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        vp_stream_copy(f.data_ptr(), g.data_ptr(), nb, stream)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 2 * f.numel() * f.element_size()
    del g
    torch.cuda.empty_cache()
    return nbytes / (ms * 1e-3) / 1e9


def code_digest(path):
    """sha256 of a C/C++/HIP source with its comments and all whitespace removed, so that
    only a change of the code itself changes it (string literals hold no comment markers
    in these sources)."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256(re.sub(r"\s+", "", text).encode()).hexdigest()


def committed_traffic(w, elem_bytes, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_hbm_traffic.md"
                        % (w.name.replace("_", ""), "f32" if elem_bytes == 4 else "f64"))
    if not os.path.exists(path):
        return None
    digests, traffic = {}, {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 3 and parts[0] == "code-sha256":
            digests[parts[2]] = parts[1]
        elif len(parts) >= 3 and parts[0] == "traffic_bytes":
            traffic[" ".join(parts[1:-1])] = float(parts[-1])
    if not digests:
        return None
    for rel, digest in digests.items():
        if code_digest(os.path.join(ROOT, rel)) != digest:
            return None
    return traffic.get(kernel)


WORKLOAD_TEXT = {
    "jeans_32x32": "Jeans instability: periodic unit cube, G=rho0=1, k/k_J=0.5, A=0.01 cosine along x on a "
                   "Maxwellian, v in [-5s,5s]^3",
    "landau_8x16": "gravitational Landau damping: periodic unit cube, G=rho0=1, k/k_J=2, A=0.05 cosine along x on a "
                   "Maxwellian, v in [-5s,5s]^3",
    "king_w6_48x48": "isolated King sphere W0=6 (G=sigma=r0=1), box +-r_t, velocities within the central escape "
                     "speed, doubled-grid Poisson",
    "slab_16x64x64_64": "one GPU's 16x64x64 slab of a 64^3 periodic box, Maxwellian (k_J=16 pi) times a Gaussian "
                        "random density field (P(k)~k^-2, rms 0.02, seed 1206), v in [-1,1]^3",
    "jeans_adjoint_16x24": "Jeans set-up with a per-cell Gaussian density perturbation (rms 1e-3, seed 6152)",
}

PHASE_KERNEL = {
    "kick": "one-pass half kick (T_vx, T_vy, T_vz of each velocity block)",
    "kick2": "one-pass pair of half kicks (two T_vz T_vy T_vx with one acceleration)",
    "drift_yz": "one-pass T_y T_z (x-slab x velocity-chunk tiles)",
    "kick_pair": "one-pass T_vz T_vy on slices of whole (vy, vz) planes",
}


def plane_slices(w, elem_bytes):
    """Planes per slice of the one-pass T_vy T_vz for cubic 48^3 and 64^3
    velocity blocks (None for other grids)."""
    nv = w.nv[0]
    if not (w.nv[1] == nv and w.nv[2] == nv and nv in (48, 64)):
        return None
    return {48: 12, 64: 8}[nv] if elem_bytes == 4 else {48: 6, 64: 4}[nv]


def x_sweep_sums(w, elem_bytes):
    """Whether the x sweep of a step also sums the density: 256 velocity cells
    per workgroup, and the workgroup's N x (256 + P) tile of new values (P the
    largest power of two up to 64 with N P <= 256) within 68 KiB of LDS."""
    nv3 = w.nv[0] * w.nv[1] * w.nv[2]
    n = w.n[0]
    p = next(q for q in (64, 32, 16, 8, 4, 2, 1) if n * q <= 256) if n <= 256 else 0
    return (nv3 % 256 == 0 and n in (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128)
            and n * (256 + p) * elem_bytes <= 68 * 1024)


def kernel_name(phase, w, elem_bytes):
    t = "float" if elem_bytes == 4 else "double"
    if phase in ("kick", "kick2"):
        if elem_bytes == 8 and tuple(w.nv) == (32, 32, 32):
            return "vp::kick_lines_f64<%d>" % (2 if phase == "kick2" else 1)
        return "vp::kick_block<%s, %d, %d, %d, %d>" % (t, w.nv[0], w.nv[1], w.nv[2], 2 if phase == "kick2" else 1)
    if phase == "kick_pair":
        return "vp::kick_pair_block<%s, %d, 2, %d>" % (t, w.nv[0], plane_slices(w, elem_bytes))
    if phase == "drift_yz":
        # (velocity cells per chunk, tiles per workgroup, chunks per cache line)
        # of the one-line-per-lane and the two-lines-per-lane kernels
        one = {16: (64, 4, 1), 24: (32, 4, 1)} if elem_bytes == 4 else {16: (32, 2, 1), 24: (16, 2, 1), 48: (8, 2, 2)}
        two = {32: (32, 4, 1), 48: (32, 4, 1), 64: (16, 4, 2)} if elem_bytes == 4 else {32: (16, 4, 1)}
        if w.n[1] in two:
            return "vp::drift_yz_pairs<%s, %d, %d, %d, %d>" % ((t, w.n[1]) + two[w.n[1]])
        return "vp::drift_yz_block<%s, %d, %d, %d, %d, %d>" % ((t, w.n[1], w.n[2]) + one[w.n[1]])
    axis = ["x", "y", "z", "vx", "vy", "vz"].index(phase)
    n = (list(w.n) + list(w.nv))[axis]
    if axis == 5:
        return "vp::sweep_contig<%s, %d>" % (t, n)
    sums = axis == 0 and x_sweep_sums(w, elem_bytes)
    return "vp::sweep_strided<%s, %d, %s>" % (t, n, "true" if sums else "false")


def gpu_run(w, vp_dtype, steps, warmup):
    import torch
    from paper_1206_6152_amd import VP_F32, Simulator, config_of
    tdt = torch.float32 if vp_dtype == VP_F32 else torch.float64
    dev = torch.device("cuda:0")
    f = build_f(w, tdt, dev)
    copy_gbps = copy_bandwidth(f)
    sim = Simulator(config_of(w, vp_dtype), f)
    e_start = sim.energy()
    # a workload without a fixed step takes the Courant step (C = 0.5) of its
    # initial state for every timed step
    dt = w.dt if w.dt > 0 else sim.dt(0.5)
    sim.run(warmup, dt)
    torch.cuda.synchronize()
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps, dt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = sim.profile_read()
    sim.profile(False)
    e_end = sim.energy()
    sim.close()
    s = f.element_size()
    cells = w.cells
    del f
    torch.cuda.empty_cache()
    per_launch = {k: (ms / n if n else 0.0) for k, (ms, n) in phases.items()}
    # candidates for the dominant kernel: single kernels (the half-block pair
    # passes of FP64 32^3 are three different kernels and are not one)
    cand = ["x", "y", "z", "vx", "vy", "vz", "kick", "kick2", "drift_yz"]
    if plane_slices(w, 4 if vp_dtype == VP_F32 else 8):
        cand.append("kick_pair")
    sweep_tot = {k: phases[k][0] for k in cand}
    dom = max(sweep_tot, key=sweep_tot.get)
    dom_ms = per_launch[dom]
    sweep_bytes = 2.0 * s * cells          # read + write f once per launch (one sweep or one fused pass)
    hbm_gbps = sweep_bytes / (dom_ms * 1e-3) / 1e9
    step_ms = wall * 1e3 / steps
    step_bytes = 19.0 * s * cells          # 9 sweeps x 2 + one density read
    # what a step of these kernels must move: every pass over f reads and writes it once
    passes = sum(n for k, (ms, n) in phases.items()
                 if k not in ("gravity", "adjoint_sweep", "adjoint_gravity", "adjoint_kick")) / max(1, steps)
    fused_bytes = passes * 2.0 * s * cells
    kname = kernel_name(dom, w, s)
    traffic = committed_traffic(w, s, kname)
    common = dict(kernel=PHASE_KERNEL.get(dom, "pfc sweep along %s" % dom), traffic=traffic,
                  traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
                  hip_kernel=kname, algorithmic_bytes_per_launch=sweep_bytes, avg_launch_ms=dom_ms,
                  hbm_GBps=hbm_gbps, hbm_frac=hbm_gbps / PEAK_HBM_GBPS)
    # the headline roofline is always HBM: the algorithmic bytes of one launch
    # (read and write f once) over its mean duration, against 8 TB/s
    roof = dict(bound="hbm", achieved=hbm_gbps, peak=PEAK_HBM_GBPS, unit="GB/s",
                frac=hbm_gbps / PEAK_HBM_GBPS, **common)
    valu = None
    if dom in ("kick", "kick2"):
        # three (or six) sweeps per pass on data held in LDS: the vector issue
        # rate is what bounds it; reported on its own, against a derived peak
        sweeps = 6 if dom == "kick2" else 3
        ops = sweeps * OPS_PER_CELL_SWEEP * cells
        tops = ops / (dom_ms * 1e-3) / 1e12
        valu = dict(achieved=tops, derived_peak=PEAK_VALU_TOPS, unit="T lane-ops/s",
                    fraction_of_derived_peak=tops / PEAK_VALU_TOPS, algorithmic_ops_per_launch=ops,
                    peak_derivation=("256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, unpacked FP32 issue "
                                     "(published 157.3 TFLOP/s / 2 for FMA / 2 for packed pairs)" if s == 4 else
                                     "256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, FP64 issue "
                                     "(published 78.6 TFLOP/s / 2 for FMA)"))
    return dict(
        value=cells * steps / wall,
        ms_per_step=step_ms,
        bytes_per_elem=s,
        dominant=dom,
        roofline=roof,
        valu=valu,
        # bytes a step of these kernels moves (every pass reads and writes f once);
        # the unfused nine-sweep model is given as an equivalent rate only
        step_model=dict(passes_per_step=passes, fused_bytes_per_step=fused_bytes,
                        fused_GBps=fused_bytes / (step_ms * 1e-3) / 1e9,
                        fused_frac=fused_bytes / (step_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                        unfused_model_bytes_per_step=step_bytes,
                        unfused_equivalent_GBps=step_bytes / (step_ms * 1e-3) / 1e9),
        phases_ms_per_launch=per_launch,
        phases_launches={k: n for k, (ms, n) in phases.items()},
        copy_GBps=copy_gbps,
        mass_drift=(e_end[2] - e_start[2]) / e_start[2],
    )


def adjoint_run():
    """The reverse mode (a8) on its own workload: vp_grad of L = -U after 40 FP32 steps of
    16^3 x 24^3 cells, checkpoint every 8 steps (forward pass, segment recomputation,
    reverse sweeps and reverse gravity), timed as one call after a warm-up call."""
    import torch
    from paper_1206_6152_amd import VP_F32, Simulator, config_of, inputs
    w = inputs.jeans_adjoint_16_24()
    k = w.params["ckpt"]
    dev = torch.device("cuda:0")
    f = build_f(w, torch.float32, dev)
    f0 = f.clone()
    sim = Simulator(config_of(w, VP_F32), f)
    sim.grad(k, w.dt, k)                      # warm-up: first launches and work buffers
    f.copy_(f0)
    sim.accel()
    torch.cuda.synchronize()
    sim.profile(True)
    t0 = time.perf_counter()
    loss, g = sim.grad(w.steps, w.dt, k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = sim.profile_read()
    sim.profile(False)
    sim.close()
    cells, s = w.cells, 4
    del f, f0, g
    torch.cuda.empty_cache()
    # the reverse kernel with the most time: the separate reverse sweeps or the
    # one-pass reverse half kicks; either reads the forward input and lam and
    # writes lam once per launch (3s bytes per cell)
    name, ms, n = max([("reverse PFC sweep (sweep_adj_kernel)",) + tuple(phases["adjoint_sweep"]),
                       ("one-pass reverse half kick (kick_adj_block)",) + tuple(phases["adjoint_kick"])],
                      key=lambda t: t[1])
    per = ms / n if n else 0.0
    rev_bytes = 3.0 * s * cells
    gbps = rev_bytes / (per * 1e-3) / 1e9 if per else 0.0
    return dict(value=cells * w.steps / wall, unit="cell-updates/s (forward steps differentiated)",
                workload=w.name, steps=w.steps, ckpt_every=k, ms_per_gradient=wall * 1e3, loss=loss,
                roofline=dict(bound="hbm", kernel=name, achieved=gbps,
                              peak=PEAK_HBM_GBPS, unit="GB/s", frac=gbps / PEAK_HBM_GBPS,
                              algorithmic_bytes_per_launch=rev_bytes, avg_launch_ms=per, launches=n),
                phases_ms={k_: v[0] for k_, v in phases.items() if v[1]})


def cpu_baseline(w, seconds):
    """The FP64 oracle, as it is, on a bounded sample of the workload: the same
    velocity grid and physics on an 8^3 spatial sub-grid, stepped for about
    `seconds` of wall time on the host's cores."""
    import numpy as np

    import oracle
    from paper_1206_6152_amd import inputs
    sub = inputs.Workload(name=w.name, n=(8, 8, 8), nv=w.nv, L=(0.25, 0.25, 0.25), vmin=w.vmin,
                          vmax=w.vmax, G=w.G, bc=w.bc, dt=w.dt, steps=1, params=w.params)
    f0 = inputs.initial_f(sub)
    g = oracle.Grid(n=sub.n, nv=sub.nv, L=sub.L, vmin=sub.vmin, vmax=sub.vmax, G=sub.G, bc=sub.bc)
    run = oracle.Run(g, f0)
    steps = 0
    t0 = time.perf_counter()
    while True:
        run.step(sub.dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    cells = sub.cells
    return dict(value=cells * steps / el, unit="cell-updates/s", cores=oracle.num_threads(),
                kind="oracle",
                sample="FP64 oracle, %d steps of an 8^3-spatial x %s-velocity sub-grid of the same "
                       "workload (%.3g cells, same Courant numbers), %.1f s wall; host %s, %d logical CPUs"
                       % (steps, "x".join(map(str, sub.nv)), cells, el, platform.processor() or
                          platform.machine(), os.cpu_count() or 0),
                cpu_model=cpu_model(), omp_num_threads=os.environ.get("OMP_NUM_THREADS"),
                single_thread=cpu_baseline_one_thread(w, max(2.0, seconds / 2)))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


_ONE_THREAD = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1206_6152_amd import inputs
w = inputs.WORKLOADS[sys.argv[2]]()
sub = inputs.Workload(name=w.name, n=(8, 8, 8), nv=w.nv, L=(0.25, 0.25, 0.25), vmin=w.vmin, vmax=w.vmax,
                      G=w.G, bc=w.bc, dt=w.dt, steps=1, params=w.params)
run = oracle.Run(oracle.Grid(n=sub.n, nv=sub.nv, L=sub.L, vmin=sub.vmin, vmax=sub.vmax, G=sub.G, bc=sub.bc),
                 inputs.initial_f(sub))
steps, t0 = 0, time.perf_counter()
while True:
    run.step(sub.dt)
    steps += 1
    el = time.perf_counter() - t0
    if el >= float(sys.argv[3]) or steps >= 50:
        break
print(json.dumps(dict(value=sub.cells * steps / el, steps=steps, wall_s=el, threads=oracle.num_threads())))
"""


def cpu_baseline_one_thread(w, seconds):
    """The same oracle sample on one host thread (OMP_NUM_THREADS=1 in a child
    process, which touches no GPU)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD, ROOT, w.name, str(seconds)], env=env,
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return dict(error=r.stderr.strip().splitlines()[-1] if r.stderr.strip() else "exit %d" % r.returncode)
    out = json.loads(r.stdout.strip().splitlines()[-1])
    out["unit"] = "cell-updates/s"
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="jeans_32x32")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-stored run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the reverse-mode measurement")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the FP32 runs of the two full-size workloads of the paper's shapes")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="profiling aid: run only the reverse-mode measurement and print it")
    ap.add_argument("--fp64-only", action="store_true",
                    help="profiling aid: run only the FP64-stored case (reported as the value, dtype f64)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the multi-GPU (x-slab) decomposition is not "
              "implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_1206_6152_amd import VP_F32, VP_F64, inputs
    w = inputs.WORKLOADS[args.workload]()
    log("workload", w.name, "cells", w.cells, "dt", w.dt)

    if args.adjoint_only:
        print(json.dumps(adjoint_run()), flush=True)
        return
    if args.fp64_only:
        r64 = gpu_run(w, VP_F64, args.steps, args.warmup)
        print(json.dumps({"metric": METRIC, "value": r64["value"], "unit": "cell-updates/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": w.name, "cells": w.cells},
                          "roofline": r64["roofline"], "step_model": r64["step_model"],
                          "phases_ms_per_launch": r64["phases_ms_per_launch"], "cpu_baseline": None}), flush=True)
        return
    r32 = gpu_run(w, VP_F32, args.steps, args.warmup)
    log("fp32", json.dumps(r32))
    r64 = None
    if not args.no_fp64:
        r64 = gpu_run(w, VP_F64, args.steps, args.warmup)
        log("fp64", json.dumps(r64))
    adj = None if args.no_adjoint else adjoint_run()
    if adj:
        log("adjoint", json.dumps(adj))
    cpu = None if args.no_cpu else cpu_baseline(w, args.cpu_seconds)
    if cpu:
        log("cpu", json.dumps(cpu))
    extra = None
    if not args.no_extra and w.name == "jeans_32x32":
        # one GPU's share of the 64^6 run and the isolated King sphere, FP32,
        # 3 timed steps each (context, not the headline value)
        extra = {}
        for name in ("slab_16x64x64_64", "king_w6_48x48"):
            wx = inputs.WORKLOADS[name]()
            rx = gpu_run(wx, VP_F32, 3, 1)
            extra[name] = {"cells": wx.cells, "ms_per_step": rx["ms_per_step"], "value": rx["value"],
                           "unit": "cell-updates/s", "passes_per_step": rx["step_model"]["passes_per_step"],
                           "fused_GBps": rx["step_model"]["fused_GBps"],
                           "dominant": {k: rx["roofline"][k] for k in ("hip_kernel", "avg_launch_ms", "achieved",
                                                                       "unit", "frac")}}
            log("extra", name, json.dumps(extra[name]))

    out = {
        "metric": METRIC,
        "value": r32["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "description": "%s; %s spatial x %s velocity cells, %s; f stored/swept in FP32, "
                           "density/Poisson/acceleration FP64"
                           % (WORKLOAD_TEXT.get(w.name, w.name), "x".join(map(str, w.n)), "x".join(map(str, w.nv)),
                              "fixed dt=%.6g" % w.dt if w.dt > 0 else "the Courant step (C=0.5) of the initial state"),
            "cells": w.cells,
            "sweeps_per_step": 9,
            "parallelism": "single GPU",
        },
        "roofline": r32["roofline"],
        "valu": r32["valu"],
        "step_model": r32["step_model"],
        "phases_ms_per_launch": r32["phases_ms_per_launch"],
        "copy_GBps": r32["copy_GBps"],
        "cpu_baseline": cpu,
        "adjoint": adj,
        "other_workloads": extra,
    }
    if r64:
        out["fp64"] = {"value": r64["value"], "ms_per_step": r64["ms_per_step"], "roofline": r64["roofline"],
                       "valu": r64["valu"], "step_model": r64["step_model"],
                       "phases_ms_per_launch": r64["phases_ms_per_launch"]}
        out["fp32_over_fp64"] = r32["value"] / r64["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
