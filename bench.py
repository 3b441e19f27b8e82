"""Benchmark of the PSTD time-step hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pstd3d|pstd2d|pstd1d|batched|...]

One bench step is one PSTD time step over the whole grid: every axis's velocity update (forward DTT,
k-space multiply with the type switch, inverse DTT, leapfrog update; one fused contraction kernel per
axis) followed by every axis's share of the pressure update.  The default workload is the 3D box of
384^3 nodes (faces drawn from the seed, c0 = 1540 m/s, CFL 0.3, FP32 state, split-bf16 contractions on
the matrix cores).  The state is resident in HBM before the timed region; the K steps replay a captured
HIP graph (captured before the timed region) between device synchronisations.

Printed: one JSON line with grid-point updates/s, the relative L2 error of the field after the
workload's full step count against the FP64 oracle's closed form, the roofline of the step (the
method's compulsory bytes over the step time measured with HIP events on the plan's stream, with the
dense design's bytes and the dominant kernel beside it), the FP64 CPU oracle timed on a bounded sample
on the host, and the batched and surrogate speedups measured in the same run outside the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp32_TFs": 157.3,
    "fp64_TFs": 78.6,
    "bf16_TFs": 2500.0,
}

WORKLOADS = {
    # name: (builder, precision, default steps, default warmup); a warmup of at least 50 steps
    # captures the plan's 50-step graph before the timed region.  Short timed regions need some tens of
    # milliseconds of warmup to reach the steady rate: after 5 steps the first 20 timed 3D steps ran 3%
    # slower, after 50 the 2049^2 FFT steps 2% slower than after 400 (200 here: that workload's accuracy is
    # taken after warmup + timed steps, and its FP32 error grows with the step count).
    "pstd2d": ("pstd2d", "fp32", 2000, 200),
    "pstd3d": ("pstd3d", "split_bf16", 50, 20),
    "pstd1d": ("pstd1d", "fp64", 1000, 100),
    "batched": ("batched", "fp32", 1000, 10),
    "faces": ("faces2d", "fp32", 1000, 300),
    "pstd2d_large": ("pstd2d_large", "fp32", 200, 200),
    "periodic2d": ("periodic2d", "fp32", 2000, 200),
    "resample3d": ("pstd3d", "split_bf16", 20, 20),
    "halfwall2d": ("halfwall2d", "fp32", 2000, 200),
    "nop": ("nop", "bf16", 20, 10),
}


# Sources of each workload's kernels and of the host code that launches them: a committed counter
# summary applies only while these files are unchanged.
SOURCES = {
    "pstd1d": ("common.h", "capi.hip", "kernels_misc.hip"),
    "pstd2d": ("common.h", "capi.hip", "kernels_phase2d.hip"),
    "pstd3d": ("common.h", "capi.hip", "tables.cpp", "structure.cpp", "kernels_split.hip"),
    "pstd2d_large": ("common.h", "capi.hip", "fft_plan.cpp", "kernels_fft.hip"),
    "periodic2d": ("common.h", "capi.hip", "tables.cpp", "kernels_phase2d.hip"),
    "resample3d": ("common.h", "capi.hip", "tables.cpp", "structure.cpp", "kernels_split.hip"),
    "halfwall2d": ("common.h", "capi.hip", "tables.cpp", "kernels_phase2d.hip"),
    "batched": ("common.h", "capi_batch.hip", "kernels_batch2d.hip"),
    "faces": ("common.h", "capi.hip", "capi_batch.hip", "kernels_batch2d.hip", "kernels_misc.hip"),
    "nop": ("common.h", "capi_nop.hip", "kernels_nop.hip"),
}


def kernel_source_hash(workload=None) -> str:
    """sha256 (first 16 hex) over the workload's kernel sources, or over all of csrc."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2005_00322_amd", "csrc")
    files = sorted(SOURCES[workload]) if workload else sorted(os.listdir(csrc))
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def fft_factorable(n):
    L = 2 * (n - 1)
    if L < 16 or L % 16:
        return False
    for f in (2, 3, 5):
        while L % f == 0:
            L //= f
    return L == 1


def uses_fft(shape, axis, precision, periodic=False):
    """Mirrors the library's automatic choice: wall-bounded axes above 512 nodes (1D: above 1365) with
    2(n-1) = 16 x 2^a 3^b 5^c run on the FFT path, and so do periodic axes of a float state whose n is a
    power of two up to 8192; other periodic axes take the dense path."""
    n = shape[axis]
    lim = 1365 if len(shape) == 1 else 512
    if periodic:
        return precision != "fp64" and lim < n <= 8192 and n & (n - 1) == 0
    cap = 8192 if precision == "fp64" else 16384
    return n > lim and fft_factorable(n) and 2 * (n - 1) <= cap


def uses_fft_velocity_launch(shape, bcs, precision):
    """Mirrors the library: when every axis of a 2D/3D float plan runs on the power-of-two FFT kernel with
    one transform length (all periodic or none), a step launches the velocity terms of all axes as one."""
    if len(shape) < 2 or precision == "fp64":
        return False
    kinds = set()
    for a, (n, (l, r)) in enumerate(zip(shape, bcs)):
        if r in (3, 4):
            return False                     # a wall half a step beyond the last node: dense path
        per = l == 2
        L = n if per else 2 * (n - 1)
        if not (uses_fft(shape, a, precision, per) and 256 <= L <= 8192 and L & (L - 1) == 0):
            return False
        kinds.add((L, per))
    return len(kinds) == 1


def uses_step1d(shape, precision, periodic):
    """Mirrors the library: 1D plans with walls on nodes, at most 1365 nodes and off the FFT path run the
    whole time loop in one workgroup (one launch per pstd_step call)."""
    return len(shape) == 1 and not periodic[0] and shape[0] <= 1365 and not uses_fft(shape, 0, precision)


def contraction_cost(shape, axis, which, precision, periodic=False):
    """Algorithmic flops and bytes of one launch along an axis.

    Dense path: 2*n_in flops per output point (a dense n_out x n_in operator applied along the axis;
    three bf16 products for split-bf16).  FFT path: 2 x 5 L log2(L) / 2 flops per line (a forward and an
    inverse complex transform of length L = 2(n-1) shared by two lines).  Bytes: the input field read
    once, the output field read and written once.  A periodic axis holds n pressure and n velocity
    points (an n x n circulant operator).
    """
    n = shape[axis]
    n_in = n if (which == 0 or periodic) else n - 1
    n_out = n if (which == 1 or periodic) else n - 1
    lines = int(np.prod(shape)) // n
    esz = 8 if precision == "fp64" else 4
    if uses_fft(shape, axis, precision, periodic):
        L = 2 * (n - 1)
        flops = 5.0 * L * np.log2(L) * lines
    else:
        flops = 2.0 * n_in * n_out * lines * (3 if precision == "split_bf16" else 1)
    bytes_ = esz * lines * (n_in + 2 * n_out)
    return flops, bytes_


def phase_cost(shape, which, precision, periodic=None):
    """Algorithmic flops and bytes of one fused phase launch (every axis at once).

    Velocity phase: every axis's contraction; p read once, each u_a read and written once.
    Pressure phase: every axis's contraction; each u_a read once, p read and written once.
    """
    periodic = periodic or [False] * len(shape)
    flops = 0.0
    esz = 8 if precision == "fp64" else 4
    pts = int(np.prod(shape))
    u_pts = [pts // n * (n if per else n - 1) for n, per in zip(shape, periodic)]
    for a in range(len(shape)):
        flops += contraction_cost(shape, a, which, precision, periodic[a])[0]
    if which == 0:
        bytes_ = esz * (pts + 2 * sum(u_pts))
    else:
        bytes_ = esz * (sum(u_pts) + 2 * pts)
    return flops, bytes_


def uses_fused_path(shape, precision):
    """Mirrors the library's automatic path choice (2D FP32 grids up to 512 x 512 use two fused kernels)."""
    return len(shape) == 2 and precision == "fp32" and max(shape) <= 512


def time_dominant_kernel(plan, st, fused, reps=50, velocity_launch=False):
    """Average duration (ms) of each kernel launch of the step, timed with events on the plan's stream.

    Keys are (axis, which); axis -1 is one launch covering every axis (a fused phase kernel, or with
    velocity_launch the FFT velocity terms of all axes).
    """
    import torch
    stream = plan._stream
    out = {}
    for which in (0, 1):
        for a in ([-1] if fused or (velocity_launch and which == 0) else range(plan.ndim)):
            plan.apply_axis(st, a, which)          # warm
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                plan.apply_axis(st, a, which)
            e1.record(stream)
            torch.cuda.synchronize()
            out[(a, which)] = e0.elapsed_time(e1) / reps
    return out


def time_fused_phases(case, precision, reps=50, replays=4):
    """Average duration (ms) of each fused phase launch, keyed (-1, which).

    A few-microsecond kernel launched back to back from the host times the host's launch rate, so `reps`
    launches of one phase are captured in a HIP graph on the plan's own stream and the graph is replayed
    on that stream between two events, as the plan's steps replay theirs.
    """
    import torch
    from paper_2005_00322_amd import Plan
    s = torch.cuda.Stream()
    out = {}
    with Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, rho0=case.rho0, precision=precision,
              stream=s) as plan:
        st = plan.new_state(case.p0)
        plan.init_state(st)
        for which in (0, 1):
            plan.apply_axis(st, -1, which)      # warm: kernel attributes set before any capture
        torch.cuda.synchronize()
        for which in (0, 1):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                for _ in range(reps):
                    plan.apply_axis(st, -1, which)
            with torch.cuda.stream(s):
                g.replay()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(replays):
                    g.replay()
                e1.record(s)
            torch.cuda.synchronize()
            out[(-1, which)] = e0.elapsed_time(e1) / (reps * replays)
            del g
    return out


def load_traffic(workload, key, src_hash, field="hbm_bytes_per_launch"):
    """HBM bytes from the committed rocprofv3 counter summary, if taken on this kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != src_hash:
        return None
    ent = rec.get("kernels", {}).get(key)
    return None if ent is None else ent.get(field)


def calibration_copies():
    """Three 256 MiB device-to-device copies: known HBM traffic for scaling the counters."""
    import torch
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cpu_baseline_leg(case, gpu_p, total_steps, budget_s=12.0):
    """The FP64 oracle on the host: time a bounded run and compare the GPU field with its closed form."""
    from threadpoolctl import threadpool_info

    from oracle import pstd as opstd

    prob = opstd.Problem(case.shape, case.bcs, case.dx, case.dt, case.c0, rho0=case.rho0)
    p = prob.project(case.p0)
    u = prob.initial_velocity(p)
    steps = 0
    t0 = time.perf_counter()
    while True:
        p, u = prob.step(p, u)
        steps += 1
        if time.perf_counter() - t0 > budget_s or steps >= case.steps:
            break
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    ref = prob.modal_solution(case.p0, total_steps)
    err = float(np.linalg.norm(gpu_p - ref) / np.linalg.norm(ref))
    base = {"value": case.points * steps / dt, "unit": "grid-point updates/s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%d of %d time steps of the same %s workload, FP64 NumPy (direct DST/DCT matrices on "
                      "wall-bounded axes, FFTs on periodic axes)"
                      % (steps, case.steps, case.name)}
    return base, err


def host_info():
    """CPU model (from /proc/cpuinfo), the cores this process may run on and the BLAS thread count."""
    from threadpoolctl import threadpool_info

    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    return model, len(os.sched_getaffinity(0)), int(threads)


def cpu_baseline_step(case, budget_s=12.0):
    """The FP64 oracle on the host at the workload's full size: the velocity half of one time step
    (u_a <- u_a - (dt/rho0) grad_a p for every axis, as the oracle's step forms it) is timed; if it
    took less than ``budget_s`` the pressure half is timed too (a whole step), otherwise the step is
    taken as twice the velocity half (the pressure half applies transforms of the same sizes)."""
    from oracle import pstd as opstd

    prob = opstd.Problem(case.shape, case.bcs, case.dx, case.dt, case.c0, rho0=case.rho0)
    p = prob.project(case.p0)
    u = [np.zeros(prob.u_shape(a)) for a in range(prob.ndim)]
    t0 = time.perf_counter()
    u_new = [u[a] - (prob.dt / prob.rho0) * prob.grad(p, a) for a in range(prob.ndim)]
    t_half = time.perf_counter() - t0
    whole = t_half < budget_s
    if whole:
        t1 = time.perf_counter()
        acc = np.zeros(prob.shape)
        for a in range(prob.ndim):
            acc += prob.div(u_new[a], a)
        p = p - prob.dt * prob.rho0 * prob.c2() * acc
        t_step = t_half + time.perf_counter() - t1
    else:
        t_step = 2.0 * t_half
    del u, u_new, p
    model, cores, threads = host_info()
    sample = ("one full time step of the %s workload at full size, FP64 NumPy (direct DST/DCT matrices), timed"
              % case.name if whole else
              "the velocity half of one time step of the %s workload at full size (three of the six transform "
              "applications), FP64 NumPy, timed; the step is taken as twice that (extrapolated)" % case.name)
    return {"value": case.points / t_step, "unit": "grid-point updates/s", "cores": cores, "blas_threads": threads,
            "cpu_model": model, "kind": "oracle", "sample": sample, "extrapolated": not whole,
            "seconds_per_step": t_step}


def step_events_ms(plan, st, n, stream):
    """Average time (ms) of one step over n steps replayed from the plan's captured graph, measured with
    HIP events on the plan's stream (the graph is captured before the first event)."""
    import torch
    plan.prepare(st, n)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    plan.step(st, n)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def headline_roofline(case, precision, step_ms, durs, src_hash, workload):
    """Roofline of the 3D step.

    The method's compulsory traffic is every state field read and written once per step: p and the
    three u_a, 4 bytes each, 8 x 4 = 32 bytes per grid point (u_a has (n_a - 1)/n_a as many points; the
    figure counts p's points).  ``achieved`` is that traffic over the step time measured with events;
    ``dense_design`` puts the six dense contractions' own bytes (input read, output read and written:
    12 bytes per point each, 72 per step) over the same time; ``dominant_kernel`` is the slowest single
    contraction launch with its algorithmic bytes over its own event-timed duration.
    """
    pts = case.points
    comp = 32.0 * pts
    gbs = comp / (step_ms * 1e-3) / 1e9
    dense = 0.0
    for a in range(len(case.shape)):
        for which in (0, 1):
            dense += contraction_cost(case.shape, a, which, precision)[1]
    dgbs = dense / (step_ms * 1e-3) / 1e9
    (axis, which), dur_ms = max(durs.items(), key=lambda kv: kv[1])
    flops, bytes_ = contraction_cost(case.shape, axis, which, precision)
    key = "axis%d_%s" % (axis, "velocity" if which == 0 else "pressure")
    kgbs = bytes_ / (dur_ms * 1e-3) / 1e9
    step_traffic = load_traffic(workload, "step", src_hash, field="hbm_bytes_per_step")
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
            "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": step_traffic,
            "launch": "one time step (the captured graph of its six contraction launches)",
            "algorithmic_bytes": int(comp), "bytes_per_point": 32, "step_ms": round(step_ms, 5),
            "dense_design": {"bytes_per_point": 72, "algorithmic_bytes": int(dense), "achieved": round(dgbs, 1),
                             "frac": round(dgbs / PEAK["hbm_GBs"], 4)},
            "dominant_kernel": {"kernel": key, "avg_ms": round(dur_ms, 5), "algorithmic_bytes": int(bytes_),
                                "algorithmic_flops": int(flops), "achieved": round(kgbs, 1),
                                "frac": round(kgbs / PEAK["hbm_GBs"], 4),
                                "mfma_tflops": round(flops / (dur_ms * 1e-3) / 1e12, 1),
                                "mfma_frac_bf16": round(flops / (dur_ms * 1e-3) / 1e12 / PEAK["bf16_TFs"], 4),
                                "traffic": load_traffic(workload, key, src_hash)}}


def run_headline(args, K, W):
    """The 3D 384^3 split-bf16 workload: K timed steps, then the batched and surrogate speedups."""
    import torch

    import workloads
    from paper_2005_00322_amd import Plan

    precision = "split_bf16"
    case = workloads.pstd3d()
    stream = torch.cuda.Stream()
    plan = Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, rho0=case.rho0, precision=precision, stream=stream)
    st = plan.new_state(case.p0)
    plan.init_state(st)
    plan.prepare(st, W)
    plan.step(st, W)
    plan.prepare(st, K)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    plan.step(st, K)
    e1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = e0.elapsed_time(e1) / K
    value = case.points * K / elapsed

    # outside the timed region: per-launch durations, the full-length accuracy run, the baselines
    durs = time_dominant_kernel(plan, st, False, reps=20)
    src_hash = kernel_source_hash("pstd3d")
    roof = headline_roofline(case, precision, step_ms, durs, src_hash, "pstd3d")
    p_final = None
    if not args.no_cpu_baseline:
        # the workload's full length from a fresh state, for the accuracy against the closed form
        st2 = plan.new_state(case.p0)
        plan.init_state(st2)
        plan.prepare(st2, case.steps)
        plan.step(st2, case.steps)
        torch.cuda.synchronize()
        p_final = st2.p.double().cpu().numpy()
        del st2
    plan.close()
    del st
    torch.cuda.empty_cache()
    err = None
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import pstd as opstd
        ref = opstd.Problem(case.shape, case.bcs, case.dx, case.dt, case.c0, rho0=case.rho0).modal_solution(
            case.p0, case.steps)
        err = float(np.linalg.norm(p_final - ref) / np.linalg.norm(ref))
        del ref
        cpu = cpu_baseline_step(case)
    del p_final
    batched = surrogate = None
    if not args.no_speedups:
        batched = batched_speedup(args)
        surrogate = surrogate_speedup(args)
    line = {
        "metric": "grid-point updates/s at stated L2 err vs FP64 oracle; batched & surrogate speedup",
        "value": value, "unit": "grid-point updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3->f32", "data": "synthetic",
        "config": {"workload": case.name, "grid": list(case.shape),
                   "bc": ["%s%s" % ("ND"[l], "ND"[r]) for l, r in case.bcs], "cfl": round(case.c0 * case.dt / case.dx, 4),
                   "precision": precision, "state": "f32", "parallelism": "single-gpu",
                   "launch": "captured HIP graph of the K steps (six split-bf16 contraction launches per step)"},
        "accuracy": {"rel_l2_vs_fp64_oracle": err, "after_steps": case.steps,
                     "reference": "FP64 discrete modal closed form of the same problem (oracle)", "tolerance": 1e-3},
        "roofline": roof, "cpu_baseline": cpu,
        "batched_speedup": batched, "surrogate_speedup": surrogate,
        "kernel_source_hash": src_hash,
    }
    print(json.dumps(line))


def batched_solves():
    import workloads
    wl = workloads.batched()
    solves, p0s, pairs, R = [], [], [], []
    for i, inst in enumerate(wl["instances"]):
        for bc in (1, 0):                       # Dirichlet then Neumann solve of each instance
            solves.append({"shape": inst.shape, "bcs": ((bc, bc), (bc, bc)), "dx": wl["dx"], "dt": inst.dt,
                           "c0": inst.c0})
            p0s.append(inst.p0)
        pairs.append((2 * i, 2 * i + 1))
        R.append(inst.R)
    return wl, solves, p0s, pairs, R


def batched_accuracy(solves, p0s, finals, combined, pairs, R, total_steps, every=16):
    """Worst relative L2 of sample solves and of their combination against the oracle's closed form."""
    from oracle import pstd as opstd

    worst = 0.0
    for k in range(0, len(pairs), every):
        d, n = pairs[k]
        refs = []
        for idx in (d, n):
            s = solves[idx]
            ref = opstd.Problem(s["shape"], s["bcs"], s["dx"], s["dt"], s["c0"]).modal_solution(p0s[idx], total_steps)
            refs.append(ref)
            worst = max(worst, float(np.linalg.norm(finals[idx] - ref) / np.linalg.norm(ref)))
        cref = opstd.combine_R(refs[0], refs[1], R[k])
        worst = max(worst, float(np.linalg.norm(combined[k] - cref) / np.linalg.norm(cref)))
    return worst


def batched_speedup(args, seq_steps=50):
    """The batched workload (128 instances x Neumann/Dirichlet = 256 uneven 2D FP32 solves, 1000 steps, one
    persistent launch from a captured graph) against the same solves run one after another through the
    single-solve FP32 path (each replaying its own captured graph on one shared stream): both timed with
    events on their streams, the single-solve path on a sample of steps of every solve."""
    import torch

    from paper_2005_00322_amd import Batch, Plan

    wl, solves, p0s, pairs, R = batched_solves()
    steps = wl["steps"] if "steps" in wl else 1000
    points = sum(s["shape"][0] * s["shape"][1] for s in solves)
    stream = torch.cuda.Stream()
    b = Batch(solves, stream=stream)
    cfg = b.autotune(trial_steps=5, cache_path=os.path.join("/tmp", "pstd_batch_tune.json"))
    st = b.new_states(p0s)
    b.init_states(st)
    b.step(st, steps)                      # warm: captures the launch graph of this step count
    b.synchronize()
    st = b.new_states(p0s)
    b.init_states(st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(st, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1)
    b.synchronize()
    outs = b.combine_R(st, pairs, R)
    torch.cuda.synchronize()
    finals = [x.p.double().cpu().numpy() for x in st]
    combined = [o.double().cpu().numpy() for o in outs]
    del st, outs
    b.close()
    # one after another: every solve on the single-solve path, graphs captured before the timed region
    seq_stream = torch.cuda.Stream()
    plans, states = [], []
    for s, p0 in zip(solves, p0s):
        pl = Plan(s["shape"], s["dx"], s["dt"], s["c0"], s["bcs"], precision="fp32", stream=seq_stream)
        x = pl.new_state(p0)
        pl.init_state(x)
        pl.prepare(x, seq_steps)
        plans.append(pl)
        states.append(x)
    torch.cuda.synchronize()
    e0.record(seq_stream)
    for pl, x in zip(plans, states):
        pl.step(x, seq_steps)
    e1.record(seq_stream)
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1) * steps / seq_steps
    for pl in plans:
        pl.close()
    del plans, states
    torch.cuda.empty_cache()
    err = None if args.no_cpu_baseline else batched_accuracy(solves, p0s, finals, combined, pairs, R, steps)
    return {"vs_sequential_single_solve_fp32": seq_ms / batched_ms, "batched_ms": batched_ms,
            "sequential_ms": seq_ms, "solves": len(solves), "steps": steps, "points_per_step": points,
            "batched_updates_per_s": points * steps / (batched_ms * 1e-3), "launch": cfg,
            "sequential_sample": "%d steps of each solve (its own captured graph, one shared stream), scaled to %d"
                                 % (seq_steps, steps),
            "accuracy": {"rel_l2_vs_fp64_oracle_worst": err, "after_steps": steps, "tolerance": 1e-5,
                         "sample": "every 16th instance: both solves and their combination"}}


def _trig_resample(n_from, n_to, kind):
    """Dense (n_to x n_from) FP64 matrix that evaluates, at the n_to equispaced nodes of the same box, the
    trigonometric series a field on n_from nodes defines: sines for Dirichlet walls at both ends (the
    type-I sine transform of the interior nodes), cosines for Neumann walls (the type-I cosine transform
    with half weights at the walls).  Modes past the smaller grid's range (and its Nyquist cosine) are
    dropped.  Measurement glue of the coarse-grid comparison (spectral interpolation between grids)."""
    N = n_from - 1
    K = min(n_from, n_to) - 1
    j = np.arange(n_from)
    t = np.arange(n_to) / (n_to - 1)                 # target positions in units of the box length
    if kind == "sine":
        k = np.arange(1, K)
        F = (2.0 / N) * np.sin(np.pi * np.outer(k, j) / N)
        F[:, 0] = F[:, -1] = 0.0
        E = np.sin(np.pi * np.outer(t, k))
    else:
        k = np.arange(0, K)
        w = np.ones(n_from)
        w[0] = w[-1] = 0.5
        F = (2.0 / N) * np.cos(np.pi * np.outer(k, j) / N) * w
        E = np.cos(np.pi * np.outer(t, k))
        E[:, 0] *= 0.5
    return E @ F


def coarse_pstd(p, c, ref, H, sizes=(64, 48, 40, 32, 24)):
    """FP32 batched PSTD of the same inputs on coarser grids over the same box and the same final time:
    p0 and the c0 map resampled spectrally onto m x m nodes, the m x m solve (its own time step at CFL
    <= 0.3 on 1600 m/s), the result evaluated back on the H x H nodes; its relative L2 error against the
    fine solver and the time of the coarse solve (events on its stream; the two resamplings are small
    GEMMs timed separately)."""
    import torch

    import workloads
    from paper_2005_00322_amd import Batch

    B = int(p.shape[0])
    L = (H - 1) * workloads.DX
    T = workloads.NOP_STEPS * workloads.NOP_DT
    out = []
    for m in sizes:
        dev = p.device
        Rx = torch.from_numpy(_trig_resample(H, m, "sine")).to(dev)      # x: Dirichlet walls
        Ry = torch.from_numpy(_trig_resample(H, m, "cosine")).to(dev)    # y: Neumann walls
        Bx = torch.from_numpy(_trig_resample(m, H, "sine")).to(dev)
        By = torch.from_numpy(_trig_resample(m, H, "cosine")).to(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(2):                     # the second pass is timed (the first loads the GEMM kernels)
            e0.record()
            pc = (Rx @ p.double() @ Ry.T).float().contiguous()
            cc = (Ry @ c.double() @ Ry.T).float().contiguous()
            e1.record()
        torch.cuda.synchronize()
        t_down = e0.elapsed_time(e1)
        dxc = L / (m - 1)
        steps = int(np.ceil(T / (0.3 * dxc / 1600.0)))
        dtc = T / steps
        cmax = cc.amax(dim=(1, 2)).double().cpu().numpy()
        solves = [{"shape": (m, m), "bcs": workloads.NOP_BCS, "dx": dxc, "dt": dtc, "c0": float(cmax[i])}
                  for i in range(B)]
        stream = torch.cuda.Stream()
        b = Batch(solves, stream=stream)
        b.set_c0_maps([cc[i] for i in range(B)])
        b.autotune(trial_steps=5, cache_path=os.path.join("/tmp", "pstd_batch_tune_coarse.json"))
        st = b.new_states([pc[i] for i in range(B)])
        b.init_states(st)
        b.step(st, steps)                      # warm: captures the launch graph of this step count
        b.synchronize()
        st = b.new_states([pc[i] for i in range(B)])
        b.init_states(st)
        torch.cuda.synchronize()
        e0.record(stream)
        b.step(st, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        t_solve = e0.elapsed_time(e1)
        b.synchronize()
        res = torch.stack([x.p for x in st]).double()
        del st
        b.close()
        e0.record()
        fine = (Bx @ res @ By.T).float()
        e1.record()
        torch.cuda.synchronize()
        t_up = e0.elapsed_time(e1)
        num = torch.linalg.vector_norm((fine - ref).double(), dim=(1, 2))
        den = torch.linalg.vector_norm(ref.double(), dim=(1, 2))
        err = (num / den).cpu().numpy()
        out.append({"grid": [m, m], "steps": steps, "solve_ms": t_solve, "resample_ms": t_down + t_up,
                    "rel_l2_vs_fp32_pstd": {"mean": float(err.mean()), "p95": float(np.quantile(err, 0.95))}})
    return out


def surrogate_speedup(args, B=256):
    """Surrogate inference on a batch of 256 held-out inputs against the batched FP32 solver on the same
    inputs (800 steps each), with the surrogate's error against that solver."""
    import torch

    import workloads
    from paper_2005_00322_amd import Batch
    from paper_2005_00322_amd.surrogate import Surrogate, SurrogateConfig

    wpath = args.weights or os.path.join(ROOT, "paper_2005_00322_amd", "weights", "nop_128x128_c32_m48_l4.npz")
    cfg = SurrogateConfig()
    p0s, c0s = workloads.nop_inputs(B, n=cfg.H, index_offset=2 * 10 ** 6)
    dev = torch.device("cuda")
    p = torch.from_numpy(p0s.astype(np.float32)).to(dev)
    c = torch.from_numpy(c0s.astype(np.float32)).to(dev)
    cmax = c.amax(dim=(1, 2)).double().cpu().numpy()
    solves = [{"shape": (cfg.H, cfg.W), "bcs": workloads.NOP_BCS, "dx": workloads.DX, "dt": workloads.NOP_DT,
               "c0": float(cmax[i])} for i in range(B)]
    stream = torch.cuda.Stream()
    b = Batch(solves, stream=stream)
    b.set_c0_maps([c[i] for i in range(B)])
    b.autotune(trial_steps=5, cache_path=os.path.join("/tmp", "pstd_batch_tune_nop.json"))
    st = b.new_states([p[i] for i in range(B)])
    b.init_states(st)
    b.step(st, workloads.NOP_STEPS)           # warm: captures the launch graph
    b.synchronize()
    st = b.new_states([p[i] for i in range(B)])
    b.init_states(st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(st, workloads.NOP_STEPS)
    e1.record(stream)
    torch.cuda.synchronize()
    pstd_ms = e0.elapsed_time(e1)
    b.synchronize()
    ref = torch.stack([x.p for x in st])
    del st
    b.close()
    net = Surrogate(cfg, max_batch=B)
    d = np.load(wpath)
    net.set_params(d["theta"])
    out = torch.empty_like(p)
    for _ in range(3):
        net.infer(p, c, out=out)
    torch.cuda.synchronize()
    reps = 10
    e0.record(net._stream)
    for _ in range(reps):
        net.infer(p, c, out=out)
    e1.record(net._stream)
    torch.cuda.synchronize()
    nop_ms = e0.elapsed_time(e1) / reps
    err = net.relative_errors(out, ref)
    net.close()
    coarse = coarse_pstd(p, c, ref, cfg.H)
    p95 = float(np.quantile(err, 0.95))
    # the cheapest coarse grid whose p95 error is at or below the surrogate's
    match = [x for x in coarse if x["rel_l2_vs_fp32_pstd"]["p95"] <= p95]
    match = min(match, key=lambda x: x["solve_ms"] + x["resample_ms"]) if match else None
    return {"vs_batched_fp32_pstd": pstd_ms / nop_ms, "pstd_ms": pstd_ms, "surrogate_ms": nop_ms, "batch": B,
            "solver_steps": workloads.NOP_STEPS, "weights": os.path.basename(wpath),
            "accuracy": {"rel_l2_vs_fp32_pstd": {"mean": float(err.mean()), "median": float(np.median(err)),
                                                 "p95": float(np.quantile(err, 0.95))},
                         "note": "errors are against the FP32 batched solver, which matches the FP64 oracle to 2e-6"},
            "coarse_pstd": coarse,
            "vs_coarse_pstd_at_matched_p95": None if match is None else {
                "grid": match["grid"], "coarse_ms": match["solve_ms"] + match["resample_ms"],
                "surrogate_ms": nop_ms, "speedup": (match["solve_ms"] + match["resample_ms"]) / nop_ms,
                "coarse_p95": match["rel_l2_vs_fp32_pstd"]["p95"], "surrogate_p95": p95}}


def batch_step_cost(solves):
    """Algorithmic flops and bytes of one step of every solve (four dense contractions per 2D step)."""
    flops = bytes_ = 0.0
    for s in solves:
        nx, ny = s["shape"]
        for which in (0, 1):
            f, b = phase_cost((nx, ny), which, "fp32")
            flops += f
            bytes_ += b
    return flops, bytes_


def run_batched(args, K, W):
    import torch

    from paper_2005_00322_amd import Batch, Plan

    wl, solves, p0s, pairs, R = batched_solves()
    points = sum(s["shape"][0] * s["shape"][1] for s in solves)
    b = Batch(solves)
    cfg = b.autotune(trial_steps=5, cache_path=os.path.join("/tmp", "pstd_batch_tune.json"))
    st = b.new_states(p0s)
    b.init_states(st)
    b.step(st, W)
    torch.cuda.synchronize()
    stream = b._stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    b.step(st, K)
    e1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = e0.elapsed_time(e1)
    outs = b.combine_R(st, pairs, R)
    torch.cuda.synchronize()
    finals = [s.p.double().cpu().numpy() for s in st]
    combined = [o.double().cpu().numpy() for o in outs]
    b.close()
    # the same solves one after another through the single-solve FP32 path (a sample of steps)
    seq_steps = 10
    seq = 0.0
    for s, p0 in zip(solves, p0s):
        with Plan(s["shape"], s["dx"], s["dt"], s["c0"], s["bcs"], precision="fp32") as pl:
            ss = pl.new_state(p0)
            pl.init_state(ss)
            pl.step(ss, 2)
            torch.cuda.synchronize()
            t = time.perf_counter()
            pl.step(ss, seq_steps)
            torch.cuda.synchronize()
            seq += time.perf_counter() - t
    seq_total = seq * K / seq_steps
    flops, bytes_ = batch_step_cost(solves)
    launches = max(1, (K + 1023) // 1024)
    tfs = flops * K / (kernel_ms * 1e-3) / 1e12
    src_hash = kernel_source_hash("batched")
    per_step = load_traffic("batched", "batch2d", src_hash, field="hbm_bytes_per_step")
    traffic = None if per_step is None else int(per_step * K / launches)
    roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": PEAK["fp32_TFs"], "unit": "TFLOP/s",
            "frac": round(tfs / PEAK["fp32_TFs"], 4), "traffic": traffic, "kernel": "batch2d_kernel (persistent)",
            "avg_ms": round(kernel_ms / launches, 3), "algorithmic_flops": int(flops * K / launches),
            "algorithmic_bytes": int(bytes_ * K / launches), "arith_intensity": round(flops / bytes_, 2)}
    cpu = err = None
    if not args.no_cpu_baseline:
        cpu, err = batched_cpu_leg(wl, solves, p0s, finals, combined, pairs, R, W + K)
    line = {
        "metric": "grid-point updates/s at stated L2 err vs FP64 oracle; batched speedup",
        "value": points * K / elapsed, "unit": "grid-point updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched2d_128x2_solves_96-512", "solves": len(solves), "points_per_step": points,
                   "precision": "fp32", "parallelism": "single-gpu", "launch": cfg},
        "batched_speedup": {"vs_sequential_single_solve_fp32": seq_total / elapsed,
                            "sequential_estimate_s": seq_total, "batched_s": elapsed,
                            "sample": "%d steps of each of the %d solves through the single-solve path, scaled to %d"
                                      % (seq_steps, len(solves), K)},
        "accuracy": {"rel_l2_vs_fp64_oracle_worst": err, "after_steps": W + K, "tolerance": 1e-5},
        "roofline": roof, "cpu_baseline": cpu, "kernel_source_hash": src_hash,
    }
    print(json.dumps(line))


def run_faces(args, K, W):
    """Per-face reflection coefficients: the 16 basic-wall solves in one batched launch plus their weighted sum."""
    import torch

    import workloads
    from paper_2005_00322_amd import Batch, combine_fields, face_weights

    case = workloads.faces2d(steps=K)
    R = case.bcs
    cases, w = face_weights(R)
    solves = [{"shape": case.shape, "bcs": cs, "dx": case.dx, "dt": case.dt, "c0": case.c0} for cs in cases]
    points = case.shape[0] * case.shape[1]
    b = Batch(solves)
    cfg = b.autotune(trial_steps=5, cache_path=os.path.join("/tmp", "pstd_batch_tune.json"))
    st = b.new_states([case.p0] * len(solves))
    b.init_states(st)
    b.step(st, W)
    out = torch.empty_like(st[0].p)
    torch.cuda.synchronize()
    stream = b._stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    b.step(st, K)
    combine_fields([s.p for s in st], w, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = e0.elapsed_time(e1)
    b.synchronize()
    got = out.double().cpu().numpy()
    b.close()
    flops, bytes_ = batch_step_cost(solves)
    # tile 16: two fused phase launches per step over all solves (the launch time here also holds the final
    # weighted sum); otherwise one persistent launch per up to 1024 steps
    phase_path = cfg.get("tile") == 16
    launches = 2 * K if phase_path else max(1, (K + 1023) // 1024)
    kernel = "phase2d_batch_kernel (velocity + pressure per step)" if phase_path else "batch2d_kernel (persistent)"
    tfs = flops * K / (kernel_ms * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": PEAK["fp32_TFs"], "unit": "TFLOP/s",
            "frac": round(tfs / PEAK["fp32_TFs"], 4), "traffic": None, "kernel": kernel,
            "avg_ms": round(kernel_ms / launches, 5), "algorithmic_flops": int(flops * K / launches),
            "algorithmic_bytes": int(bytes_ * K / launches), "arith_intensity": round(flops / bytes_, 2)}
    cpu = err = None
    if not args.no_cpu_baseline:
        cpu, err = faces_cpu_leg(case, got, W + K)
    line = {
        "metric": "grid-point updates/s at stated L2 err vs FP64 oracle",
        "value": points * K / elapsed, "unit": "grid-point updates/s (of the per-face-R field)", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": case.name, "grid": list(case.shape), "R_faces": [list(r) for r in R],
                   "basic_solves": len(solves), "basic_updates_per_s": points * len(solves) * K / elapsed,
                   "precision": "fp32", "parallelism": "single-gpu", "launch": cfg},
        "accuracy": {"rel_l2_vs_fp64_oracle": err, "after_steps": W + K, "tolerance": 1e-5},
        "roofline": roof, "cpu_baseline": cpu, "kernel_source_hash": kernel_source_hash("faces"),
    }
    print(json.dumps(line))


def resample_cost(shape, axis, which, precision):
    """Algorithmic flops and bytes of one launch of a collocated-derivative / interpolation operator along
    an axis: a dense n_out x n_in operator per line (three bf16 products for split-bf16), the input read
    once and the output written once."""
    n = shape[axis]
    n_in = n if which in (2, 4) else n - 1
    n_out = n if which in (2, 5) else n - 1
    lines = int(np.prod(shape)) // n
    esz = 8 if precision == "fp64" else 4
    flops = 2.0 * n_in * n_out * lines * (3 if precision == "split_bf16" else 1)
    return flops, esz * lines * (n_in + n_out)


def run_resample(args, K, W):
    """Velocity output on the pressure grid (§3.4): the three particle-velocity fields of the 384^3
    split-bf16 3D workload resampled half a step onto the nodes, one launch per axis."""
    import torch

    import workloads
    from paper_2005_00322_amd import STAG_TO_NODES, Plan

    case = workloads.pstd3d()
    prec = "split_bf16"
    plan = Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, rho0=case.rho0, precision=prec)
    st = plan.new_state(case.p0)
    plan.init_state(st)
    plan.step(st, 2)
    outs = [torch.empty(case.shape, device="cuda", dtype=torch.float32) for _ in range(3)]

    def one():
        for a in range(3):
            plan.apply_operator(a, STAG_TO_NODES, st.u[a], outs[a])

    for _ in range(max(W, 1)):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        one()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = 3 * case.points * K / elapsed

    # per-axis launch durations with events on the plan's stream
    stream = plan._stream
    durs = {}
    for a in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            plan.apply_operator(a, STAG_TO_NODES, st.u[a], outs[a])
        e1.record(stream)
        torch.cuda.synchronize()
        durs[a] = e0.elapsed_time(e1) / 10
    axis, dur_ms = max(durs.items(), key=lambda kv: kv[1])
    flops, bytes_ = resample_cost(case.shape, axis, STAG_TO_NODES, prec)
    gbs = bytes_ / (dur_ms * 1e-3) / 1e9
    tfs = flops / (dur_ms * 1e-3) / 1e12
    src_hash = kernel_source_hash("resample3d")
    key = "axis%d_stag_to_nodes" % axis
    traffic = load_traffic("resample3d", key, src_hash)
    ridge = PEAK["bf16_TFs"] * 1e12 / (PEAK["hbm_GBs"] * 1e9)
    if flops / bytes_ < ridge:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": traffic}
    else:
        roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": PEAK["bf16_TFs"], "unit": "TFLOP/s",
                "frac": round(tfs / PEAK["bf16_TFs"], 4), "traffic": traffic}
    roof.update({"kernel": key, "avg_ms": round(dur_ms, 5), "algorithmic_bytes": int(bytes_),
                 "algorithmic_flops": int(flops), "arith_intensity": round(flops / bytes_, 2)})

    # accuracy: 64 sampled lines of each output against the oracle's interpolation of the same input lines
    u_host = [u.double().cpu().numpy() for u in st.u]
    got = [o.double().cpu().numpy() for o in outs]
    plan.close()
    cpu = err = None
    if not args.no_cpu_baseline:
        cpu, err = resample_cpu_leg(case, u_host, got)
    line = {
        "metric": "grid-point updates/s at stated L2 err vs FP64 oracle",
        "value": value, "unit": "velocity values resampled onto the nodes /s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": elapsed / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3->f32", "data": "synthetic",
        "config": {"workload": "resample3d_384^3_u_to_nodes", "grid": list(case.shape),
                   "bc": ["%s%s" % ("ND"[l], "ND"[r]) for l, r in case.bcs], "operator": "staggered -> nodes",
                   "precision": prec, "parallelism": "single-gpu"},
        "accuracy": {"rel_l2_vs_fp64_oracle_sampled_lines": err, "lines": "64 per axis (32 of largest energy, 32 random)",
                     "tolerance": 1e-3},
        "roofline": roof, "cpu_baseline": cpu, "kernel_source_hash": src_hash,
    }
    print(json.dumps(line))


def resample_cpu_leg(case, u_host, got, budget_s=12.0):
    """The oracle's interpolation (FP64 NumPy) on whole planes of lines: times as many planes as fit the
    budget and compares 64 sampled GPU lines per axis with it."""
    from threadpoolctl import threadpool_info

    from oracle import pstd as opstd

    rng = np.random.default_rng(5)
    worst = 0.0
    done = 0
    for a in range(3):
        # the 32 lines of largest energy and 32 random ones; relative L2 over all of them (far from the
        # pulses a line holds only values below the field's FP32 resolution)
        ax = opstd.Axis(case.shape[a], case.bcs[a][0], case.bcs[a][1], case.dx)
        um = np.moveaxis(u_host[a], a, -1)
        gm = np.moveaxis(got[a], a, -1)
        energy = np.einsum("ijk,ijk->ij", um, um)
        top = np.argsort(energy, axis=None)[-32:]
        picks = [divmod(int(t), um.shape[1]) for t in top]
        picks += [tuple(int(v) for v in rng.integers(0, um.shape[:2])) for _ in range(32)]
        num = den = 0.0
        for i, j in picks:
            ref = ax.interp_u_to_p(um[i, j])
            num += float(np.sum((gm[i, j] - ref) ** 2))
            den += float(np.sum(ref ** 2))
        worst = max(worst, float(np.sqrt(num / den)))
    t0 = time.perf_counter()
    planes = 0
    while time.perf_counter() - t0 < budget_s and planes < case.shape[0]:
        for a in range(3):
            ax = opstd.Axis(case.shape[a], case.bcs[a][0], case.bcs[a][1], case.dx)
            um = np.moveaxis(u_host[a], a, -1)
            ax.interp_u_to_p(um[planes])
            done += um.shape[1] * case.shape[a]
        planes += 1
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    base = {"value": done / dt, "unit": "velocity values resampled onto the nodes /s", "cores": int(threads),
            "kind": "oracle",
            "sample": "%d of %d planes of lines of each of the three velocity fields, FP64 NumPy (forward "
                      "transform, inverse of the other symmetry)" % (planes, case.shape[0])}
    return base, worst


def faces_cpu_leg(case, got, total_steps, budget_s=12.0):
    """Oracle: the 16 basic solves stepped on the host for a bounded time; the GPU field against the
    weighted sum of the basic fields' FP64 closed forms."""
    from threadpoolctl import threadpool_info

    from oracle import pstd as opstd

    ws = opstd.combination_weights(case.bcs)
    probs = [(opstd.Problem(case.shape, cs, case.dx, case.dt, case.c0), wi) for cs, wi in ws.items()]
    pu = [(pr.project(case.p0), pr.initial_velocity(case.p0)) for pr, _ in probs]
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < total_steps:
        pu = [pr.step(p, u) for (pr, _), (p, u) in zip(probs, pu)]
        steps += 1
    dt = time.perf_counter() - t0
    threads = max([x.get("num_threads", 1) for x in threadpool_info() if x.get("user_api") == "blas"] or [1])
    ref = sum(wi * pr.modal_solution(case.p0, total_steps) for pr, wi in probs)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    pts = case.shape[0] * case.shape[1]
    cpu = {"value": pts * steps / dt, "unit": "grid-point updates/s (of the per-face-R field)", "cores": threads,
           "kind": "oracle", "sample": "%d of %d time steps of all 16 basic solves, FP64 NumPy" % (steps, total_steps)}
    return cpu, err


def batched_cpu_leg(wl, solves, p0s, finals, combined, pairs, R, total_steps, budget_s=12.0):
    """Oracle: time stepping of sample solves on the host; check sample solves and combinations."""
    from threadpoolctl import threadpool_info

    from oracle import pstd as opstd

    # timing sample: the first solves, stepped until the budget is used
    done_pts = 0
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < budget_s and i < len(solves):
        s = solves[i]
        prob = opstd.Problem(s["shape"], s["bcs"], s["dx"], s["dt"], s["c0"])
        p, u = prob.project(p0s[i]), prob.initial_velocity(p0s[i])
        n = 0
        while n < 50 and time.perf_counter() - t0 < budget_s:
            p, u = prob.step(p, u)
            n += 1
        done_pts += n * s["shape"][0] * s["shape"][1]
        i += 1
    dt = time.perf_counter() - t0
    threads = max([x.get("num_threads", 1) for x in threadpool_info() if x.get("user_api") == "blas"] or [1])
    # accuracy: every 16th instance, both solves and their combination, against the closed form
    worst = 0.0
    for k in range(0, len(pairs), 16):
        d, n = pairs[k]
        refs = []
        for idx in (d, n):
            s = solves[idx]
            ref = opstd.Problem(s["shape"], s["bcs"], s["dx"], s["dt"], s["c0"]).modal_solution(p0s[idx], total_steps)
            refs.append(ref)
            worst = max(worst, float(np.linalg.norm(finals[idx] - ref) / np.linalg.norm(ref)))
        cref = opstd.combine_R(refs[0], refs[1], R[k])
        worst = max(worst, float(np.linalg.norm(combined[k] - cref) / np.linalg.norm(cref)))
    cpu = {"value": done_pts / dt, "unit": "grid-point updates/s", "cores": int(threads), "kind": "oracle",
           "sample": "up to 50 time steps of the first %d solves of the batched workload, FP64 NumPy" % i}
    return cpu, worst


def nop_forward_flops(H, W, C, Mm, layers, Hp):
    """Multiply-add flops (x2) of one surrogate forward pass per sample (the GEMMs of the network)."""
    P = H * W
    per_layer = 2 * C * (Mm * H * W + Mm * Mm * W)        # DCT along H, then along W
    per_layer += 2 * Mm * Mm * C * C                     # per-mode channel mixing
    per_layer += 2 * C * (Mm * Mm * W + Mm * H * W)      # inverse along W, then along H
    per_layer += 2 * C * C * P                           # pointwise channel mixing
    return layers * per_layer + 2 * P * (4 * C + C * Hp + Hp)


def nop_forward_bytes(H, W, C, Mm, layers, B):
    """Algorithmic HBM bytes of one surrogate forward: every tensor the network materialises (the lifted
    field, each layer's output, each layer's DCT coefficients and mixed coefficients) written once and
    read once, plus the two input fields read and the output written; FP32 throughout."""
    act = 4 * B * C * H * W
    spec = 4 * B * C * Mm * Mm
    return (layers + 1) * 2 * act + layers * 2 * 2 * spec + 3 * 4 * B * H * W


def run_nop(args, K, W):
    """Surrogate inference (batch 256) against the batched FP32 solver on the same 256 held-out inputs."""
    import torch

    import workloads
    from paper_2005_00322_amd import Batch
    from paper_2005_00322_amd.surrogate import Surrogate, SurrogateConfig

    wpath = args.weights or os.path.join(ROOT, "paper_2005_00322_amd", "weights", "nop_128x128_c32_m48_l4.npz")
    cfg = SurrogateConfig()
    B = 256
    p0s, c0s = workloads.nop_inputs(B, n=cfg.H, index_offset=2 * 10 ** 6)
    dev = torch.device("cuda")
    p = torch.from_numpy(p0s.astype(np.float32)).to(dev)
    c = torch.from_numpy(c0s.astype(np.float32)).to(dev)
    # the solver: 256 solves x 800 steps in one batched launch sequence (timed region: the steps only)
    cmax = c.amax(dim=(1, 2)).double().cpu().numpy()
    solves = [{"shape": (cfg.H, cfg.W), "bcs": workloads.NOP_BCS, "dx": workloads.DX, "dt": workloads.NOP_DT,
               "c0": float(cmax[i])} for i in range(B)]
    b = Batch(solves)
    b.set_c0_maps([c[i] for i in range(B)])
    b.autotune(trial_steps=5, cache_path=os.path.join("/tmp", "pstd_batch_tune_nop.json"))
    st = b.new_states([p[i] for i in range(B)])
    b.init_states(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(st, workloads.NOP_STEPS)
    torch.cuda.synchronize()
    t_pstd = time.perf_counter() - t0
    ref = torch.stack([s.p for s in st])
    b.close()
    # the surrogate
    net = Surrogate(cfg, max_batch=B)
    d = np.load(wpath)
    net.set_params(d["theta"])
    out = torch.empty_like(p)
    for _ in range(W):
        net.infer(p, c, out=out)
    torch.cuda.synchronize()
    stream = net._stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(K):
        net.infer(p, c, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    t_nop = (time.perf_counter() - t0) / K
    ev_ms = e0.elapsed_time(e1) / K
    err = net.relative_errors(out, ref)
    net.close()
    pts = cfg.H * cfg.W
    flops = nop_forward_flops(cfg.H, cfg.W, cfg.channels, cfg.modes, cfg.layers, cfg.hidden) * B
    bytes_ = nop_forward_bytes(cfg.H, cfg.W, cfg.channels, cfg.modes, cfg.layers, B)
    tfs = flops / (ev_ms * 1e-3) / 1e12
    gbs = bytes_ / (ev_ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_info

        from oracle import nop as onop
        ocfg = onop.Config()
        theta = d["theta"].astype(np.float64)
        t0 = time.perf_counter()
        ns = 0
        while ns < 2:
            onop.forward(ocfg, theta, p0s[ns:ns + 1], c0s[ns:ns + 1])
            ns += 1
        tcpu = time.perf_counter() - t0
        threads = max([x.get("num_threads", 1) for x in threadpool_info() if x.get("user_api") == "blas"] or [1])
        cpu = {"value": ns * pts * workloads.NOP_STEPS / tcpu, "unit": "equivalent grid-point updates/s",
               "cores": int(threads), "kind": "oracle",
               "sample": "FP64 NumPy surrogate forward of %d of the 256 samples (einsum contractions)" % ns}
    line = {
        "metric": "grid-point updates/s at stated L2 err vs FP64 oracle; surrogate speedup",
        "value": B * pts * workloads.NOP_STEPS / t_nop, "unit": "equivalent grid-point updates/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": t_nop * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
        "config": {"workload": "nop_128x128_batch256_t800", "grid": [cfg.H, cfg.W], "channels": cfg.channels,
                   "modes": cfg.modes, "layers": cfg.layers, "hidden": cfg.hidden, "batch": B,
                   "solver_steps": workloads.NOP_STEPS, "weights": os.path.basename(wpath),
                   "trained_pairs": int(d["train"]), "trained_epochs": int(d["epochs"]), "parallelism": "single-gpu"},
        "accuracy": {"rel_l2_vs_fp32_pstd": {"mean": float(err.mean()), "median": float(np.median(err)),
                                             "p95": float(np.quantile(err, 0.95))},
                     "note": "errors are against the FP32 batched solver, which matches the FP64 oracle to 2e-6"},
        "surrogate_speedup": {"vs_batched_fp32_pstd": t_pstd / t_nop, "pstd_s": t_pstd, "surrogate_s": t_nop,
                              "sample": "the same 256 inputs, %d steps each" % workloads.NOP_STEPS},
        # flops / bytes is about 33, far below the bf16 ridge (2500 / 8 = 312): bound by HBM
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                     "frac": round(gbs / PEAK["hbm_GBs"], 4),
                     "traffic": load_traffic("nop", "forward", kernel_source_hash("nop"), field="hbm_bytes_per_forward"),
                     "kernel": "one inference forward (all its kernels)",
                     "avg_ms": round(ev_ms, 4), "algorithmic_bytes": int(bytes_), "algorithmic_flops": int(flops),
                     "arith_intensity": round(flops / bytes_, 2), "mfma_frac_bf16": round(tfs / PEAK["bf16_TFs"], 5)},
        "cpu_baseline": cpu, "kernel_source_hash": kernel_source_hash("nop"),
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="pstd3d", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-speedups", action="store_true",
                    help="pstd3d: skip the batched and surrogate speedup measurements")
    ap.add_argument("--weights", default=None, help="surrogate parameters (npz with 'theta') for --workload nop")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run three 256 MiB device-to-device copies (known HBM traffic, for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads
    from paper_2005_00322_amd import Plan

    builder, precision, dsteps, dwarm = WORKLOADS[args.workload]
    K = dsteps if args.steps is None else args.steps
    W = dwarm if args.warmup is None else args.warmup
    if args.calibrate_copy:
        torch.cuda.set_device(0)
        calibration_copies()
    if args.workload == "pstd3d":
        torch.cuda.set_device(0)
        run_headline(args, K, W)
        return
    if args.workload == "faces":
        torch.cuda.set_device(0)
        run_faces(args, K, W)
        return
    if args.workload == "batched":
        torch.cuda.set_device(0)
        run_batched(args, K, W)
        return
    if args.workload == "resample3d":
        torch.cuda.set_device(0)
        run_resample(args, K, W)
        return
    if args.workload == "nop":
        torch.cuda.set_device(0)
        run_nop(args, K, W)
        return
    case = getattr(workloads, builder)()
    torch.cuda.set_device(0)

    plan = Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, rho0=case.rho0, precision=precision)
    st = plan.new_state(case.p0)
    plan.init_state(st)
    plan.step(st, W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(st, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    p_final = st.p.double().cpu().numpy()
    value = case.points * K / elapsed

    # dominant kernel: the single contraction launch with the largest average duration
    # axes with n staggered points: periodic, or a right wall half a step beyond the last node
    periodic = [l == 2 or r in (3, 4) for l, r in case.bcs]
    fused = uses_fused_path(case.shape, precision)
    if uses_step1d(case.shape, precision, periodic):
        # one workgroup runs the whole time loop: its two matrix-vector products per step are FP64
        # vector FMAs on one CU (operators held in registers or streamed from L2, the state in LDS), so
        # the bound is that CU's FP64 vector rate and no HBM traffic is made per step
        n = case.shape[0]
        flops = 4.0 * n * (n - 1)
        step_ms = elapsed / K * 1e3
        peak_cu = PEAK["fp64_TFs"] / 256
        tfs = flops / (step_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(tfs, 5), "peak": round(peak_cu, 4), "unit": "TFLOP/s",
                "frac": round(tfs / peak_cu, 4), "traffic": None,
                "kernel": "step1d (one launch for all steps; per step)", "avg_ms": round(step_ms, 6),
                "algorithmic_bytes": 0, "algorithmic_flops": int(flops),
                "peak_basis": "FP64 vector FMA rate of one CU (78.6 TFLOP/s / 256 CUs)"}
        plan.close()
        cpu = err = None
        if not args.no_cpu_baseline:
            cpu, err = cpu_baseline_leg(case, p_final, W + K)
        print(json.dumps(single_grid_line(case, precision, value, K, W, elapsed, err, roof, cpu,
                                          kernel_source_hash(args.workload))))
        return
    vel_fft = uses_fft_velocity_launch(case.shape, case.bcs, precision)
    if fused:
        durs = time_fused_phases(case, precision)
    else:
        state_copy = plan.new_state(case.p0)
        plan.init_state(state_copy)
        durs = time_dominant_kernel(plan, state_copy, fused, velocity_launch=vel_fft)
    (axis, which), dur_ms = max(durs.items(), key=lambda kv: kv[1])
    if axis < 0:
        flops, bytes_ = phase_cost(case.shape, which, precision, periodic)
    else:
        flops, bytes_ = contraction_cost(case.shape, axis, which, precision, periodic[axis])
    gbs = bytes_ / (dur_ms * 1e-3) / 1e9
    tfs = flops / (dur_ms * 1e-3) / 1e12
    peak_c = {"fp32": PEAK["fp32_TFs"], "fp64": PEAK["fp64_TFs"], "split_bf16": PEAK["bf16_TFs"]}[precision]
    fft_launch = (axis >= 0 and uses_fft(case.shape, axis, precision, periodic[axis])) or (axis < 0 and vel_fft)
    if fft_launch:
        peak_c = PEAK["fp64_TFs"] if precision == "fp64" else PEAK["fp32_TFs"]   # FFT butterflies: vector ALU
    ai = flops / bytes_
    ridge = peak_c * 1e12 / (PEAK["hbm_GBs"] * 1e9)
    src_hash = kernel_source_hash(args.workload)
    key = ("all_axes" if axis < 0 and vel_fft else "fused" if axis < 0 else "axis%d" % axis) + "_" + \
        ("velocity" if which == 0 else "pressure")
    if fft_launch:
        key += "_fft"
    traffic = load_traffic(args.workload, key, src_hash)
    if ai < ridge:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": round(gbs / PEAK["hbm_GBs"], 4), "traffic": traffic}
    else:
        roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": peak_c, "unit": "TFLOP/s",
                "frac": round(tfs / peak_c, 4), "traffic": traffic}
    roof.update({"kernel": key, "avg_ms": round(dur_ms, 5), "algorithmic_bytes": int(bytes_),
                 "algorithmic_flops": int(flops), "arith_intensity": round(ai, 2)})
    plan.close()
    cpu = None
    err = None
    if not args.no_cpu_baseline:
        cpu, err = cpu_baseline_leg(case, p_final, W + K)

    print(json.dumps(single_grid_line(case, precision, value, K, W, elapsed, err, roof, cpu, src_hash)))


def single_grid_line(case, precision, value, K, W, elapsed, err, roof, cpu, src_hash):
    """The JSON line of a single-grid workload."""
    dtype = {"fp32": "f32", "fp64": "f64", "split_bf16": "bf16x3->f32"}[precision]
    return {
        "metric": "grid-point updates/s at stated L2 err vs FP64 oracle",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": case.name, "grid": list(case.shape),
                   "bc": ["%s%s" % (("N", "D", "P", "Nh", "Dh")[l], ("N", "D", "P", "Nh", "Dh")[r]) for l, r in case.bcs], "cfl": round(case.c0 * case.dt / case.dx, 4),
                   "precision": precision, "parallelism": "single-gpu"},
        "accuracy": {"rel_l2_vs_fp64_oracle": err, "after_steps": W + K,
                     "tolerance": {"fp32": 1e-5, "fp64": 1e-10, "split_bf16": 1e-3}[precision]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_source_hash": src_hash,
    }


if __name__ == "__main__":
    main()
