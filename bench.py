"""Throughput of the TDSE propagation hot path on one MI355X.

A step of this benchmark is one whole propagation of the Lmax=15, N=500
single-instance workload (8000 complex128 states, 20-cycle pulse, RK4 with
dt=0.005: 50266 time steps, 201064 dipole products). The metric is
state-steps/s = states x time steps / wall time, with inputs resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line. `roofline` describes the dominant kernel (the fused
tile kernel, one launch per dipole product); `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 matrix / vector


METRIC = "state-steps/s (matvec % HBM peak; batched % FP64 MFMA) at 1e-10 vs oracle"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_vec_tiles_L15_N500.json")
# sources that determine the tile kernel's code (and so its traffic and trace)
TILE_KERNEL_SOURCES = ["vec_kernels.hip", "tdse_vec.h", "tdse_split.h", "tdse_tile.h", "tdse_reduce.h"]


def tile_kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TILE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1201_6062_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per tile-kernel launch from the committed FETCH_SIZE / WRITE_SIZE
    measurement, or None when the kernel sources changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != tile_kernel_hash():
        return None
    return t.get("bytes_per_launch")


TRACE_FILE = os.path.join(ROOT, "profiles", "trace_vec_tiles_L15_N500.json")


def traced_launch_us():
    """Average vec_tiles_kernel dispatch duration (us) from the committed
    rocprofv3 kernel trace of this benchmark, or None when the kernel sources
    changed since it was taken."""
    if not os.path.exists(TRACE_FILE):
        return None
    with open(TRACE_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != tile_kernel_hash():
        return None
    return t.get("avg_us")


def algorithmic_bytes_per_product(lmax: int, n: int) -> int:
    """Dipole read once (8 L N^2) + energies (8 n) + one complex vector in and out (32 n)."""
    ns = (lmax + 1) * n
    return 8 * lmax * n * n + 40 * ns


def time_propagation(plan, w, method, order, steps, warmup, torch):
    import torch as _t
    f = _t.as_tensor(w.field, device="cuda")
    c0 = _t.as_tensor(w.c0, device="cuda")
    out = _t.empty_like(c0)
    for _ in range(warmup):
        plan.propagate(f, c0, w.dt, method, order=order, out=out)
    _t.cuda.synchronize()
    stream = _t.cuda.current_stream()
    e0, e1 = _t.cuda.Event(enable_timing=True), _t.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.propagate(f, c0, w.dt, method, order=order, out=out)
    e1.record(stream)
    _t.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_s = e0.elapsed_time(e1) / 1e3
    return ev_s, wall, out.cpu().numpy()


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo) and the cores this job may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    nproc = os.cpu_count() or 1
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    # the job's CPU share: OMP_NUM_THREADS is set to it where the job runs
    share = int(os.environ.get("OMP_NUM_THREADS", nproc) or nproc)
    return model, nproc, max(1, min(nproc, share))


def cpu_worker(pulse_index: int, nsteps: int):
    """One single-threaded oracle run (child process of the all-core baseline):
    the first nsteps RK4 steps of pulse pulse_index of the 256-pulse set on the
    Lmax=15, N=500 Hamiltonian. Prints its wall time."""
    import oracle
    from paper_1201_6062_amd import workloads as wl
    h = wl.hamiltonian(15, 500, 0)
    p = wl.random_pulses(np.random.default_rng(1), 256)[pulse_index]
    f = wl.rk4_samples(p, 0.005, nsteps)[None]
    c0 = wl.ground_state(15, 500)
    t = time.perf_counter()
    oracle.rk4(h.energies, h.dipole, 0.005, f, c0)
    print(json.dumps({"seconds": time.perf_counter() - t}), flush=True)


def cpu_baseline(w, target_s: float = 15.0):
    """The oracle on the host cores: one thread on the first steps of the
    benchmark workload, and every core of the job's share at once, each
    running its own pulse (independent pulses on the same Hamiltonian, the
    way the batched workloads parallelise), as child processes."""
    import subprocess
    import oracle
    oracle.build(force=False)
    h = w.ham

    def run(k):
        if w.method == "rk4":
            oracle.rk4(h.energies, h.dipole, w.dt, w.field[:, :k], w.c0)
        else:
            oracle.taylor(h.energies, h.dipole, w.order, w.dt, w.field[:, :k], w.c0)
    # size the sample from one timed step
    t = time.perf_counter()
    run(1)
    per = time.perf_counter() - t
    nst = max(1, min(w.nsteps, int(target_s / max(per, 1e-6))))
    t = time.perf_counter()
    run(nst)
    el = time.perf_counter() - t
    single = h.nstates * nst / el
    model, nproc, cores = host_cpu()
    # all cores: `cores` child processes, each one thread on its own pulse
    nst_all = max(1, nst // 2)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    t = time.perf_counter()
    try:
        procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(i), str(nst_all)],
                                  stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, env=env) for i in range(cores)]
        outs = [p.communicate()[0] for p in procs]
        ok = all(p.returncode == 0 for p in procs)
    except OSError:
        ok = False
    wall = time.perf_counter() - t
    per_proc = [json.loads(o.decode().strip().splitlines()[-1])["seconds"] for o in outs] if ok else []
    allcore = h.nstates * nst_all * cores / wall if ok else None
    return {"value": allcore if ok else single, "unit": "state-steps/s", "cores": cores if ok else 1,
            "kind": "oracle",
            "sample": (f"{cores} single-threaded oracle processes at once, each the first {nst_all} RK4 steps of its "
                       f"own pulse (pulses 0..{cores - 1} of the 256-pulse set) on the Lmax=15 N=500 Hamiltonian, "
                       f"{wall:.1f} s wall" if ok else
                       f"first {nst} of {w.nsteps} steps of the workload, one thread, {el:.1f} s"),
            "single_core": {"value": single, "cores": 1,
                            "sample": f"first {nst} of {w.nsteps} {w.method} steps of the Lmax=15 N=500 workload, "
                                      f"one thread, {el:.1f} s"},
            "all_core_per_process_s": per_proc,
            "host": {"cpu_model": model, "nproc": nproc, "cores_used": cores if ok else 1},
            "paper_context": "the paper reports about 40x for its OpenCL code on an AMD FirePro V7800 over one core "
                             "of a Xeon W3503 (Taylor-10, FP64, its own basis; Sec. 5.1, Fig. GPURUNTIME): "
                             "context, not a target"}


def hbm_diagnostic(torch, steps=64):
    """Lmax=63, N=1000 (504 MB of dipole, far beyond L2 and MALL): HBM-streaming rate."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    lmax, n, dt = 63, 1000, 0.005
    en = wl.energies(lmax, n)
    rng = np.random.default_rng(5)
    dip = rng.standard_normal((lmax, n, n)) * 0.01
    plan = Plan(en, dip)
    f = wl.rk4_samples(wl.Pulse(0.05, 0.5, 20.0), dt, steps)[None]
    c0 = wl.ground_state(lmax, n)

    class W:
        pass
    w = W()
    w.field, w.c0, w.dt = f, c0, dt
    ev, _, _ = time_propagation(plan, w, "rk4", 0, 3, 1, torch)
    per_launch = ev / 3 / (4 * steps)
    b = algorithmic_bytes_per_product(lmax, n)
    plan.close()
    return {"workload": "Lmax=63 N=1000 RK4, 64 steps", "bytes_per_product": b,
            "us_per_product": per_launch * 1e6, "GBps": b / per_launch / 1e9,
            "frac_of_hbm_peak": b / per_launch / 1e9 / HBM_PEAK_GBS}


def batched_measure(torch, batch: int = 256, steps: int = 100, tile: str | None = None):
    """256 pulses on the Lmax=15 N=500 Hamiltonian (RK4 dt=0.005): FP64 matrix-core rate."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    if tile:
        os.environ["TDSE_TILE"] = tile
    w = wl.batched(batch)
    plan = Plan(w.ham.energies, w.ham.dipole, batch=batch)
    if tile:
        del os.environ["TDSE_TILE"]
    f = torch.as_tensor(np.ascontiguousarray(w.field[:, :steps]), device="cuda")
    c0 = torch.as_tensor(w.c0, device="cuda")
    plan.propagate(f[:, :2], c0, w.dt, "rk4")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.propagate(f, c0, w.dt, "rk4")
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    lmax, n = w.ham.lmax, w.ham.n
    flop_stage = 8.0 * lmax * n * n * batch
    tf = flop_stage * 4 * steps / s / 1e12
    plan.close()
    return {"workload": f"{batch} pulses, Lmax=15 N=500, RK4 dt=0.005, first {steps} of {w.nsteps} steps",
            "state_steps_per_s": w.ham.nstates * batch * steps / s,
            "us_per_stage": s / (4 * steps) * 1e6, "flop_per_stage": flop_stage,
            "tflops": tf, "frac_of_fp64_peak": tf / FP64_PEAK_TFLOPS}


def small_measure(torch, force_tiles: bool = False):
    """Lmax=3, N=50 (200 states), 12567 RK4 steps: the latency-bound small problem."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    w = wl.single_small()
    if force_tiles:
        os.environ["TDSE_TILE"] = "T=1"
    plan = Plan(w.ham.energies, w.ham.dipole)
    if force_tiles:
        del os.environ["TDSE_TILE"]
    ev, _, _ = time_propagation(plan, w, "rk4", 0, 3, 1, torch)
    plan.close()
    t = ev / 3
    return {"workload": "Lmax=3 N=50, RK4 dt=0.01, 12567 steps", "path": "tiles" if force_tiles else "one workgroup",
            "ms_per_propagation": t * 1e3, "state_steps_per_s": w.ham.nstates * w.nsteps / t,
            "us_per_step": t / w.nsteps * 1e6}


def taylor8_measure(torch):
    """Lmax=15, N=500 with Taylor-8, dt=0.02 (12567 steps, 100536 products): the
    second propagator the single-instance workload is run with."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    w = wl.single_large("taylor", 8)
    plan = Plan(w.ham.energies, w.ham.dipole)
    ev, _, cT = time_propagation(plan, w, "taylor", 8, 2, 1, torch)
    plan.close()
    t = ev / 2
    err = None
    gold = os.path.join(ROOT, "tests", "golden", "single_large_taylor8.npz")
    if os.path.exists(gold):
        g = np.load(gold, allow_pickle=False)["cT"]
        err = float(np.linalg.norm(cT[0] - g) / np.linalg.norm(g))
    bpp = algorithmic_bytes_per_product(15, 500)
    per = t / (8 * w.nsteps)
    return {"workload": "Lmax=15 N=500, Taylor-8 dt=0.02, 12567 steps", "s_per_propagation": t,
            "state_steps_per_s": w.ham.nstates * w.nsteps / t, "us_per_product": per * 1e6,
            "GBps": bpp / per / 1e9, "frac_of_hbm_peak": bpp / per / 1e9 / HBM_PEAK_GBS,
            "max_rel_err_vs_oracle": err}


def lanczos_measure(torch, m: int = 12, dt: float = 0.05, steps: int = 256, batch: int = 1):
    """Lmax=15, N=500 short-iterative Lanczos (Krylov dimension m, midpoint
    samples); batch > 1: that many pulses of one Hamiltonian (c3's pulse
    distribution), the batched product."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    h = wl.hamiltonian(15, 500, 0)
    plan = Plan(h.energies, h.dipole, batch=batch)
    if batch == 1:
        fs = wl.taylor_samples(wl.Pulse(0.05, 0.5, 20.0), dt, steps, "mid")[None]
    else:
        fs = np.stack([wl.taylor_samples(p, dt, steps, "mid") for p in wl.random_pulses(np.random.default_rng(1), batch)])
    f = torch.as_tensor(fs, device="cuda")
    c0 = torch.as_tensor(wl.ground_state(15, 500, batch), device="cuda")
    plan.propagate(f[:, :64], c0, dt, "lanczos", order=m)  # warm-up, captures the 64-step chunk graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.propagate(f, c0, dt, "lanczos", order=m)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    plan.close()
    what = "the 20-cycle pulse" if batch == 1 else f"{batch} pulses"
    return {"workload": f"Lmax=15 N=500, Lanczos m={m}, dt={dt}, first {steps} steps of {what}",
            "state_steps_per_s": h.nstates * batch * steps / s, "us_per_step": s / steps * 1e6,
            "us_per_product": s / (steps * m) * 1e6}


def lmax_sweep(torch, n: int = 500, steps: int = 512):
    """Per-product time of the fused tile kernel against the dipole size at
    N=500: flat while the dipole fits the XCDs' L2 (launch-latency floor),
    then a step where it stops fitting."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    out = []
    for lmax in (7, 11, 13, 15, 16, 17, 19, 23):
        en = wl.energies(lmax, n)
        dip = np.random.default_rng(lmax).standard_normal((lmax, n, n)) * 0.01
        plan = Plan(en, dip)

        class W:
            pass
        w = W()
        w.field = wl.rk4_samples(wl.Pulse(0.05, 0.5, 20.0), 0.005, steps)[None]
        w.c0, w.dt = wl.ground_state(lmax, n), 0.005
        ev, _, _ = time_propagation(plan, w, "rk4", 0, 3, 1, torch)
        plan.close()
        us = ev / 3 / (4 * steps) * 1e6
        mb = 8 * lmax * n * n / 1e6
        out.append({"lmax": lmax, "dipole_MB": mb, "MB_per_xcd": mb / 8, "us_per_product": us,
                    "GBps": algorithmic_bytes_per_product(lmax, n) / us / 1e3})
    return {"workload": "fused tile kernel, N=500, RK4, 512 steps per size", "points": out}


def group_measure(torch, steps: int = 400, reps: int = 1):
    """64 uneven instances (Lmax 7..31, N 200..1000), first `steps` RK4 steps
    of each (the fastest of `reps` timed calls)."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Group, Plan
    specs = wl.uneven_specs(64)
    plans, fs, cs = [], [], []
    for sp in specs:
        h = wl.hamiltonian(sp.lmax, sp.n, sp.seed)
        plans.append(Plan(h.energies, h.dipole))
        fs.append(torch.as_tensor(wl.rk4_samples(sp.pulse, 0.005, min(steps, sp.nsteps)), device="cuda"))
        cs.append(torch.as_tensor(wl.ground_state(sp.lmax, sp.n)[0], device="cuda"))
    g = Group(plans)
    g.propagate(fs, cs, 0.005)  # untimed: captures the chunk graphs the timed call replays
    torch.cuda.synchronize()
    s = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.propagate(fs, cs, 0.005)
        e1.record()
        torch.cuda.synchronize()
        s = min(s, e0.elapsed_time(e1) / 1e3)
    nbytes = sum(4 * f.shape[0] * algorithmic_bytes_per_product(sp.lmax, sp.n) for sp, f in zip(specs, fs))
    ss = sum((sp.lmax + 1) * sp.n * f.shape[0] for sp, f in zip(specs, fs))
    g.close()
    for p in plans:
        p.close()
    return {"workload": f"64 instances (Lmax 7..31, N 200..1000, {sum(sp.lmax * sp.n ** 2 * 8 for sp in specs) / 1e9:.2f} GB "
                        f"of dipole), first {steps} RK4 steps each", "seconds": s,
            "state_steps_per_s": ss / s, "GBps": nbytes / s / 1e9, "frac_of_hbm_peak": nbytes / s / 1e9 / HBM_PEAK_GBS}


def rkf45_measure(torch, batch: int = 256, steps: int = 50):
    """256 pulses on the Lmax=15 N=500 Hamiltonian, Runge-Kutta-Fehlberg 4(5)
    with per-step error estimates (six stages per step), dt=0.005."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    h, dt = wl.hamiltonian(15, 500, 0), 0.005
    plan = Plan(h.energies, h.dipole, batch=batch)
    pulses = wl.random_pulses(np.random.default_rng(1), batch)
    f = torch.as_tensor(np.stack([wl.rkf45_samples(p, dt, steps) for p in pulses]), device="cuda")
    c0 = torch.as_tensor(wl.ground_state(15, 500, batch), device="cuda")
    plan.propagate_rkf45(f[:, :2], c0, dt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.propagate_rkf45(f, c0, dt)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    flop_stage = 8.0 * h.lmax * h.n * h.n * batch
    tf = flop_stage * 6 * steps / s / 1e12
    plan.close()
    return {"workload": f"{batch} pulses, Lmax=15 N=500, RKF 4(5) with error estimates, dt={dt}, {steps} steps",
            "state_steps_per_s": h.nstates * batch * steps / s, "us_per_stage": s / (6 * steps) * 1e6,
            "tflops": tf, "frac_of_fp64_peak": tf / FP64_PEAK_TFLOPS}


def velocity_measure(torch, steps: int = 2048):
    """The single-instance workload in the velocity gauge (coupling A(t) P,
    P = -i Q): RK4 dt=0.005 on the first `steps` steps of the 20-cycle pulse."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    h = wl.hamiltonian(15, 500, 0)
    q = wl.velocity_coupling(h.energies, h.dipole)
    plan = Plan(h.energies, q, gauge="velocity")
    f = torch.as_tensor(wl.vector_potential_samples(wl.Pulse(0.05, 0.5, 20.0), 0.005, steps)[None], device="cuda")
    c0 = torch.as_tensor(wl.ground_state(15, 500), device="cuda")
    plan.propagate(f[:, :64], c0, 0.005, "rk4")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.propagate(f, c0, 0.005, "rk4")
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    per = s / (4 * steps)
    bpp = algorithmic_bytes_per_product(15, 500)
    plan.close()
    return {"workload": f"Lmax=15 N=500 velocity gauge, RK4 dt=0.005, first {steps} steps",
            "state_steps_per_s": h.nstates * steps / s, "us_per_product": per * 1e6,
            "GBps": bpp / per / 1e9, "frac_of_hbm_peak": bpp / per / 1e9 / HBM_PEAK_GBS}


def adjoint_measure(torch, steps: int = 2048, method: str = "rk4", order: int = 8):
    """The adjoint workload (32 pulses of piecewise-constant samples on the
    Lmax=15 N=500 Hamiltonian, RK4 dt=0.01, checkpoints every 64 steps), first
    `steps` steps: forward with checkpoints, then the reverse sweep (segment
    recompute + adjoint stages). FP64 matrix-core rate over all 12 stages per
    step. method="taylor": the same samples through the Taylor series of
    `order` (3 * order products per step: forward, recompute, adjoint)."""
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan
    h = wl.hamiltonian(15, 500, 0)
    pulses = wl.adjoint_pulses(32)
    spi = wl.ADJ_STEPS_PER_INTERVAL
    ek = np.stack([wl.piecewise_samples(p) for p in pulses])[:, : max(1, steps // spi)]
    slots = 3 if method == "rk4" else 1
    f = torch.as_tensor(wl.expand_piecewise(ek, spi, slots), device="cuda")
    nsteps = f.shape[1]
    c0 = torch.as_tensor(wl.ground_state(15, 500, 32), device="cuda")
    dt, batch = 0.01, 32
    plan = Plan(h.energies, h.dipole, batch=batch)
    en = torch.as_tensor(plan.energies, device="cuda")
    mask = (en > 0).to(torch.float64).repeat_interleave(2)
    kw = dict(method=method, order=order)
    cT, ck = plan.propagate(f[:, :64], c0, dt, ckpt_every=64, **kw)  # warm-up
    plan.adjoint(f[:, :64], c0, dt, 2.0 * cT * mask[None, :], ckpt=ck, ckpt_every=64, **kw)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    cT, ck = plan.propagate(f, c0, dt, ckpt_every=64, **kw)
    ev[1].record()
    g, l0 = plan.adjoint(f, c0, dt, 2.0 * cT * mask[None, :], ckpt=ck, ckpt_every=64, **kw)
    ev[2].record()
    torch.cuda.synchronize()
    tf, tb = ev[0].elapsed_time(ev[1]) / 1e3, ev[1].elapsed_time(ev[2]) / 1e3
    flop_stage = 8.0 * h.lmax * h.n * h.n * batch
    per_step = 4 if method == "rk4" else order
    stages = 3 * per_step * nsteps  # forward, recompute and adjoint products
    tflops = flop_stage * stages / (tf + tb) / 1e12
    plan.close()
    name = "RK4" if method == "rk4" else f"Taylor-{order}"
    return {"workload": f"{batch} pulses, Lmax=15 N=500, {name} dt=0.01, piecewise-constant field, checkpoints "
                        f"every 64 steps, first {nsteps} of {wl.ADJ_INTERVALS * spi} steps",
            "forward_s": tf, "reverse_s": tb, "reverse_over_forward": tb / tf,
            "state_steps_per_s": h.nstates * batch * nsteps / (tf + tb),
            "flop_per_stage": flop_stage, "tflops": tflops, "frac_of_fp64_peak": tflops / FP64_PEAK_TFLOPS}


def tuned_measure(torch, group_steps: int = 400):
    """The autotuner on the adjoint workload's shape (Lmax=15, N=500, 32
    pulses: a forward RK4 stage) and on the 64 uneven instances (each shape
    tuned alone, then the group run on its tuned tile counts), each against
    the library's default tiles."""
    import tempfile
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan, tune
    out = {}
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.json")
        t = time.perf_counter()
        msg = tune(15, 500, 32, cache)
        tune_s = time.perf_counter() - t
        h = wl.hamiltonian(15, 500, 0)
        pulses = wl.adjoint_pulses(32)
        f = torch.as_tensor(np.stack([wl.rk4_samples(p, 0.01, 256) for p in pulses]), device="cuda")
        c0 = torch.as_tensor(wl.ground_state(15, 500, 32), device="cuda")

        def stage_us():
            # a whole untimed propagation first (graph capture), then the
            # fastest of three timed ones
            plan = Plan(h.energies, h.dipole, batch=32)
            plan.propagate(f, c0, 0.01, "rk4")
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                plan.propagate(f, c0, 0.01, "rk4")
                e1.record()
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1) * 1e3 / (4 * f.shape[1]))
            plan.close()
            return best
        default_us = stage_us()
        os.environ["TDSE_TUNE_CACHE"] = cache
        try:
            tuned_us = stage_us()
        finally:
            del os.environ["TDSE_TUNE_CACHE"]
        out["adjoint_shape_B32"] = {"tuner": msg, "tune_s": tune_s, "default_us_per_stage": default_us,
                                    "tuned_us_per_stage": tuned_us, "tuned_over_default_speed": default_us / tuned_us}
        t = time.perf_counter()
        for sp in wl.uneven_specs(64):
            tune(sp.lmax, sp.n, 1, cache)
        tune_s = time.perf_counter() - t
        with open(cache) as fh:
            ent = json.load(fh)["entries"]
        # (T = 0 in the cache: the tuner kept the library's own choice)
        moved = [sp for sp in wl.uneven_specs(64)
                 if ent[f"L{sp.lmax}_N{sp.n}_B1"]["T"] not in (0, (sp.n + 127) // 128)]

        def lone_s(sp, steps=256):
            # one instance on its own: an untimed call, then the faster of two
            h = wl.hamiltonian(sp.lmax, sp.n, sp.seed)
            f = torch.as_tensor(wl.rk4_samples(sp.pulse, 0.005, steps), device="cuda")[None]
            c0 = torch.as_tensor(wl.ground_state(sp.lmax, sp.n), device="cuda")
            plan = Plan(h.energies, h.dipole)
            plan.propagate(f, c0, 0.005, "rk4")
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(2):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                plan.propagate(f, c0, 0.005, "rk4")
                e1.record()
                torch.cuda.synchronize()
                best = min(best, e0.elapsed_time(e1) / 1e3)
            plan.close()
            return best
        lone_default = sum(lone_s(sp) for sp in moved)
        default = group_measure(torch, steps=group_steps, reps=2)
        os.environ["TDSE_TUNE_CACHE"] = cache
        try:
            lone_tuned = sum(lone_s(sp) for sp in moved)
            tuned = group_measure(torch, steps=group_steps, reps=2)
        finally:
            del os.environ["TDSE_TUNE_CACHE"]
        out["uneven_group"] = {"tune_s": tune_s, "instances_off_default_tiles": len(moved),
                               "alone_tuned_over_default_speed": lone_default / lone_tuned if moved else 1.0,
                               "alone_note": "those instances propagated one at a time (256 RK4 steps each), "
                                             "summed: where the tuned tile counts apply",
                               "default_frac_of_hbm_peak": default["frac_of_hbm_peak"],
                               "tuned_frac_of_hbm_peak": tuned["frac_of_hbm_peak"],
                               "tuned_over_default_speed": tuned["GBps"] / default["GBps"],
                               "group_note": "a group streams every member at its default tile count "
                                             "(re-tiled copies of the tuned members' blocks)"}
    return out


def library_references(torch, reps: int = 20):
    """What vendor library code reaches on this GPU, beside the kernels' own
    fractions: FP64 batched GEMMs of the batched stage's shape (16 blocks,
    512 x 1024 by 1024 x 2B: the products of one RK4 stage without the
    epilogue, at 256 and at 32 pulses) through torch.bmm (rocBLAS /
    hipBLASLt), and a 1 GiB device-to-device copy (bytes read + written)."""
    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps
    g = torch.Generator(device="cuda").manual_seed(0)
    gemm = {}
    for cols in (512, 64):  # 256 pulses; 32 pulses (the adjoint workload)
        a = torch.randn(16, 512, 1024, dtype=torch.float64, device="cuda", generator=g)
        b = torch.randn(16, 1024, cols, dtype=torch.float64, device="cuda", generator=g).contiguous()
        c = torch.empty(16, 512, cols, dtype=torch.float64, device="cuda")
        s = timed(lambda: torch.bmm(a, b, out=c))
        gemm[cols] = 2.0 * 16 * 512 * cols * 1024 / s / 1e12
        del a, b, c
    x = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    s = timed(lambda: y.copy_(x))
    tbs = 2.0 * x.numel() * 8 / s / 1e12
    del x, y
    return {"fp64_bmm": {"what": "torch.bmm FP64, 16 x (512x1024 @ 1024x512)", "tflops": gemm[512],
                         "frac_of_fp64_peak": gemm[512] / FP64_PEAK_TFLOPS},
            "fp64_bmm_64_columns": {"what": "torch.bmm FP64, 16 x (512x1024 @ 1024x64)", "tflops": gemm[64],
                                    "frac_of_fp64_peak": gemm[64] / FP64_PEAK_TFLOPS},
            "device_copy": {"what": "1 GiB FP64 tensor copy_ (read + write)", "TBps": tbs,
                            "frac_of_hbm_peak": tbs * 1e3 / HBM_PEAK_GBS}}


def calibrate_copy(torch, mb: int = 1024, reps: int = 5):
    """Plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    x = torch.ones(mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_MiB": mb, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-diag", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the small-problem and group measurements")
    ap.add_argument("--only", choices=["single", "diag", "batched", "small", "small_tiles", "group", "taylor8",
                                       "lanczos", "lanczos_b8", "lsweep", "adjoint", "adjoint_taylor8", "rkf45",
                                       "velocity", "tuned", "refs"],
                    default=None,
                    help="profiling runs: measure one workload and print its record alone")
    ap.add_argument("--tile", default=None, help="batched tile TMxTN (tuning experiments)")
    ap.add_argument("--method", choices=["rk4", "taylor"], default="rk4")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--truncate", type=int, default=0,
                    help="profiling runs only: propagate the first STEPS time steps")
    ap.add_argument("--cpu-worker", nargs=2, type=int, default=None, metavar=("PULSE", "NSTEPS"),
                    help="internal: one single-threaded oracle run of the all-core CPU baseline")
    a = ap.parse_args()
    if a.cpu_worker:
        cpu_worker(*a.cpu_worker)
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(each pulse batch would run on its own GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # The CPU baseline runs first, before this process touches the GPU (its
    # all-core leg starts child processes).
    cpu = None
    if a.only is None and not a.no_cpu_baseline and not a.calibrate_copy:
        from paper_1201_6062_amd import workloads as wl0
        w0 = wl0.single_large(a.method, 8)
        if a.truncate:
            w0.nsteps = min(w0.nsteps, a.truncate)
            w0.field = np.ascontiguousarray(w0.field[:, : w0.nsteps])
        cpu = cpu_baseline(w0)

    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    if a.calibrate_copy:
        calibrate_copy(torch)
        return
    from paper_1201_6062_amd import workloads as wl
    from paper_1201_6062_amd.api import Plan

    only = {"diag": lambda: hbm_diagnostic(torch),
            "batched": lambda: batched_measure(torch, steps=a.truncate or 100, tile=a.tile),
            "small": lambda: small_measure(torch),
            "small_tiles": lambda: small_measure(torch, force_tiles=True),
            "group": lambda: group_measure(torch, steps=a.truncate or 400),
            "taylor8": lambda: taylor8_measure(torch),
            "lanczos": lambda: lanczos_measure(torch),
            "lanczos_b8": lambda: lanczos_measure(torch, batch=8, steps=64),
            "lsweep": lambda: lmax_sweep(torch),
            "adjoint": lambda: adjoint_measure(torch, steps=a.truncate or 2048),
            "adjoint_taylor8": lambda: adjoint_measure(torch, steps=a.truncate or 512, method="taylor", order=8),
            "rkf45": lambda: rkf45_measure(torch, steps=a.truncate or 50),
            "velocity": lambda: velocity_measure(torch),
            "tuned": lambda: tuned_measure(torch),
            "refs": lambda: library_references(torch)}
    if a.only in only:
        print(json.dumps(only[a.only]()))
        return
    w = wl.single_large(a.method, 8)
    if a.truncate:
        w.nsteps = min(w.nsteps, a.truncate)
        w.field = np.ascontiguousarray(w.field[:, : w.nsteps])
    plan = Plan(w.ham.energies, w.ham.dipole)
    ev_s, wall_s, cT = time_propagation(plan, w, a.method, 8, a.steps, a.warmup, torch)
    ns = w.ham.nstates
    products_per_step = 4 if a.method == "rk4" else 8
    launches = w.nsteps * products_per_step
    ms_per_step = ev_s / a.steps * 1e3
    value = ns * w.nsteps * a.steps / ev_s
    per_launch = ev_s / a.steps / launches
    bpp = algorithmic_bytes_per_product(w.ham.lmax, w.ham.n)

    err = None
    gold = os.path.join(ROOT, "tests", "golden", f"single_large_{'rk4' if a.method == 'rk4' else 'taylor8'}.npz")
    if os.path.exists(gold) and not a.truncate:
        g = np.load(gold, allow_pickle=False)["cT"]
        err = float(np.linalg.norm(cT[0] - g) / np.linalg.norm(g))

    traffic = measured_traffic()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "state-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded hydrogen-like Hamiltonian and sin^2 pulse)",
        "config": {"workload": f"single instance Lmax=15 N=500 (8000 states), "
                               f"{'RK4 dt=0.005' if a.method == 'rk4' else 'Taylor-8 dt=0.02'}, "
                               f"20-cycle pulse E0=0.05 w=0.5, {w.nsteps} time steps per propagation",
                   "states": ns, "time_steps": w.nsteps, "products_per_propagation": launches},
        "roofline": {"bound": "hbm", "achieved": bpp / per_launch / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": bpp / per_launch / 1e9 / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": "vec_tiles_kernel", "bytes_per_launch": bpp,
                     "us_per_launch": per_launch * 1e6,
                     "us_per_launch_timing": "HIP events over the timed propagations on the launch stream, "
                                             "divided by the product launches: start to start, so it includes "
                                             "the gaps between launches and the per-chunk staging kernels",
                     "limited_by": "launch latency, not HBM: the 30 MB dipole stays in the XCDs' L2 across "
                                   "launches (3.75 MB per XCD of 4 MB); about 2.3 us of each launch is the "
                                   "kernel boundary. The HBM-streaming rates are in hbm_streaming",
                     "traffic_note": "FETCH_SIZE + WRITE_SIZE per dispatch under rocprofv3 --pmc, where "
                                     "dispatches run serialized and start with a cold L2: an upper bound of "
                                     "the steady-state HBM traffic"},
        "max_rel_err_vs_oracle": err,
        "wall_s_host": wall_s,
    }
    tr = traced_launch_us()
    out["roofline"]["us_per_launch_traced"] = tr
    out["roofline"]["frac_traced"] = bpp / (tr * 1e-6) / 1e9 / HBM_PEAK_GBS if tr else None
    out["roofline"]["trace_profile"] = os.path.relpath(TRACE_FILE, ROOT) if tr else None
    plan.close()
    if a.only == "single":
        print(json.dumps(out))
        return
    hs = {}
    if not a.no_diag:
        out["hbm_diagnostic"] = hbm_diagnostic(torch)
        hs["beyond_cache_diagnostic"] = {"workload": out["hbm_diagnostic"]["workload"],
                                         "frac": out["hbm_diagnostic"]["frac_of_hbm_peak"],
                                         "note": "504 MB of dipole, twice the 256 MB memory-side cache (MALL); "
                                                 "successive products stream in opposite directions, so part "
                                                 "of each launch's first tiles come from the MALL: algorithmic "
                                                 "bytes over time, not bytes the HBM delivered"}
    if not a.no_batched:
        out["batched"] = batched_measure(torch)
        out["library_references"] = library_references(torch)
    if not a.no_extra:
        out["single_small"] = small_measure(torch)
        out["single_small_tiles"] = small_measure(torch, force_tiles=True)
        out["uneven_group"] = group_measure(torch)
        hs["uneven_group"] = {"workload": out["uneven_group"]["workload"],
                              "frac": out["uneven_group"]["frac_of_hbm_peak"]}
        out["single_taylor8"] = taylor8_measure(torch)
        out["lanczos"] = lanczos_measure(torch)
        out["lanczos_8_pulses"] = lanczos_measure(torch, batch=8, steps=64)
        out["adjoint"] = adjoint_measure(torch)
        out["adjoint_taylor8"] = adjoint_measure(torch, steps=512, method="taylor", order=8)
        out["rkf45"] = rkf45_measure(torch)
        out["velocity_gauge"] = velocity_measure(torch)
        out["autotuner"] = tuned_measure(torch)
    out["roofline"]["hbm_streaming"] = hs or None
    if cpu is not None:
        out["cpu_baseline"] = cpu
        out["cpu_baseline"]["gpu_over_cpu"] = value / cpu["value"]
        out["cpu_baseline"]["gpu_over_single_core"] = value / cpu["single_core"]["value"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
