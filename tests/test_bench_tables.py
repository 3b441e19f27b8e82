"""Host checks of bench.py's workload tables and cost model (no GPU)."""
import subprocess
import sys

import numpy as np

import bench
import workloads


def test_every_workload_has_sources_and_builder():
    for name, (builder, precision, steps, warmup) in bench.WORKLOADS.items():
        assert name in bench.SOURCES, name
        assert precision in ("fp32", "fp64", "split_bf16", "bf16")
        assert steps > 0 and warmup >= 0
        if builder not in ("batched", "nop"):
            assert callable(getattr(workloads, builder)), builder
        assert len(bench.kernel_source_hash(name)) == 16
    for fn in ("faces_cpu_leg", "batched_cpu_leg", "resample_cpu_leg", "cpu_baseline_leg", "run_faces",
               "run_batched", "run_nop", "run_resample", "time_fused_phases"):
        assert callable(getattr(bench, fn)), fn


def test_cost_model_staggered_extents():
    n = 64
    # wall-bounded: velocity reads n, writes n-1 points per line; periodic / half-step wall: n and n
    f0, b0 = bench.contraction_cost((n, n), 1, 0, "fp32")
    assert f0 == 2.0 * n * (n - 1) * n and b0 == 4 * n * (n + 2 * (n - 1))
    f1, b1 = bench.contraction_cost((n, n), 1, 0, "fp32", periodic=True)
    assert f1 == 2.0 * n * n * n and b1 == 4 * n * 3 * n
    f, b = bench.phase_cost((n, n), 1, "fp32", [True, False])
    assert b == 4 * ((n * n + n * (n - 1)) + 2 * n * n)
    f, b = bench.resample_cost((n, n, n), 2, 5, "split_bf16")
    assert f == 2.0 * (n - 1) * n * n * n * 3 and b == 4 * n * n * ((n - 1) + n)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_fft_velocity_launch_mirror():
    # the library launches the velocity terms of all axes together when every axis runs on the
    # power-of-two FFT kernel with one transform length (all periodic or none)
    N, D, P, Nh = 0, 1, 2, 3
    f = bench.uses_fft_velocity_launch
    assert f((2049, 2049), ((D, D), (N, N)), "fp32")
    assert f((1025, 1025, 1025), ((N, N), (D, N), (N, D)), "split_bf16")
    assert f((1024, 1024), ((P, P), (P, P)), "fp32")
    assert not f((2049, 2049), ((D, D), (N, N)), "fp64")         # FP64: mixed-radix kernel
    assert not f((2049,), ((D, N),), "fp32")                       # 1D: one axis
    assert not f((2049, 1025), ((D, D), (N, N)), "fp32")          # two transform lengths
    assert not f((2049, 400), ((D, D), (N, N)), "fp32")           # a dense axis
    assert not f((1024, 513), ((P, P), (N, D)), "fp32")           # periodic beside walls
    assert not f((2049, 2049), ((D, D), (N, Nh)), "fp32")         # a half-step wall: dense
    assert not f((1537, 1537), ((D, D), (N, N)), "fp32")          # L = 3072: mixed-radix kernel
