"""GPU parity of the FP32 FFT kernel specialised to power-of-two transform lengths (2(n-1) = 256 .. 8192).

Each case applies the velocity and the pressure term along every such axis once, on unit-stride
(contiguous) and strided axes and on every pair of wall types, and compares with the FP64 oracle's DTT
recipe element by element (FP32 bound 2e-6, as for the mixed-radix kernel) and with the mixed-radix
kernel on the same input (the two agree to the same bound and differ in rounding, so both ran).  Periodic
axes of n = 256 .. 8192 points (a power of two: the transform is the line itself) are compared with the
oracle's Fourier recipe and, up to 4096 points, with the dense contraction.
"""
import numpy as np
import pytest

from gpu_helpers import rel_l2
from oracle import pstd as opstd

pytestmark = pytest.mark.gpu
N, D = opstd.NEUMANN, opstd.DIRICHLET

CASES = [
    ((129, 40), ((N, D), (D, N))),
    ((40, 129), ((D, D), (N, N))),
    ((257, 33), ((D, N), (N, N))),
    ((24, 513), ((N, N), (D, N))),
    ((1025, 12), ((D, D), (N, D))),
    ((12, 2049), ((N, D), (D, D))),
    ((2049, 10), ((N, N), (D, D))),
    ((4097, 6), ((D, N), (N, N))),
    ((6, 4097), ((N, N), (N, D))),
    ((129, 20, 257), ((D, N), (N, N), (N, D))),
]


P = opstd.PERIODIC


def _pow2_axis(n):
    L = 2 * (n - 1)
    return 256 <= L <= 8192 and L & (L - 1) == 0


@pytest.mark.parametrize("shape,bcs", CASES)
def test_pow2_kernel_vs_oracle_and_mixed_radix(shape, bcs):
    import torch
    from paper_2005_00322_amd import Plan

    print("case", shape, bcs, flush=True)
    dx, c0 = 1e-3, 1500.0
    dt = 0.25 * dx / c0
    prob = opstd.Problem(shape, bcs, dx, dt, c0)
    rng = np.random.default_rng(sum(shape))
    p = prob.project(rng.standard_normal(shape))
    axes = [a for a in range(len(shape)) if _pow2_axis(shape[a])]
    assert axes
    results = {}
    for path in ("fft", "fft_generic"):
        with Plan(shape, dx, dt, c0, bcs, precision="fp32") as plan:
            plan.set_path(path)
            for a in axes:
                u = rng.standard_normal(prob.u_shape(a)) if path == "fft" else results[("u_in", a)]
                results[("u_in", a)] = u
                st = plan.new_state(p)
                for b in range(len(shape)):
                    st.u[b].zero_()
                plan.apply_axis(st, a, 0)
                torch.cuda.synchronize()
                results[(path, a, 0)] = st.u[a].double().cpu().numpy()
                st = plan.new_state(np.zeros(shape))
                st.u[a].copy_(torch.from_numpy(u).to(st.u[a].dtype))
                plan.apply_axis(st, a, 1)
                torch.cuda.synchronize()
                results[(path, a, 1)] = st.p.double().cpu().numpy()
    for a in axes:
        refs = (-(dt / prob.rho0) * prob.grad(p, a), -(dt * prob.rho0 * c0 ** 2) * prob.div(results[("u_in", a)], a))
        for which in (0, 1):
            got, other = results[("fft", a, which)], results[("fft_generic", a, which)]
            e = rel_l2(got, refs[which])
            print("axis", a, "which", which, "rel_l2", e, "vs mixed radix", rel_l2(got, other), flush=True)
            assert e < 2e-6
            assert rel_l2(other, refs[which]) < 2e-6
            assert not np.array_equal(got, other)


def test_pow2_kernel_steps_with_c0_map():
    # a few full steps of a 2D problem with a heterogeneous medium (the pressure epilogue's per-point
    # factor) on both kernels, against the oracle's run of the same steps
    import workloads
    from gpu_helpers import oracle_problem, run_gpu

    rng = np.random.default_rng(5)
    shape = (257, 129)
    dx, c0 = 1e-3, 1500.0
    c0_map = workloads.smooth_c0_map(rng, shape)
    dt = 0.25 * dx / float(c0_map.max())
    p0 = workloads.gaussian(shape, dx, (100 * dx, 60 * dx), 6 * dx)
    case = workloads.Case("pow2_map", shape, ((D, N), (N, D)), dx, dt, float(c0_map.max()), 40, p0, c0_map=c0_map)
    # the device sees the float32 map
    case32 = workloads.Case("pow2_map", shape, case.bcs, dx, dt, case.c0, 40, p0,
                            c0_map=c0_map.astype(np.float32).astype(np.float64))
    ref_p, _ = oracle_problem(case32).run(p0, case.steps)
    got, _ = run_gpu(case, precision="fp32", path="fft")
    gen, _ = run_gpu(case, precision="fp32", path="fft_generic")
    print("rel_l2 pow2", rel_l2(got, ref_p), "mixed radix", rel_l2(gen, ref_p), flush=True)
    assert rel_l2(got, ref_p) < 1e-5
    assert rel_l2(gen, ref_p) < 1e-5


PERIODIC_CASES = [
    ((256, 24), ((P, P), (D, N))),
    ((20, 1024), ((N, D), (P, P))),
    ((2048, 8), ((P, P), (N, N))),
    ((8, 4096), ((D, D), (P, P))),
    ((8192, 4), ((P, P), (D, D))),
]


@pytest.mark.parametrize("shape,bcs", PERIODIC_CASES)
def test_pow2_kernel_periodic_axes(shape, bcs):
    import torch
    from paper_2005_00322_amd import Plan

    print("case", shape, bcs, flush=True)
    dx, c0 = 1e-3, 1500.0
    dt = 0.25 * dx / c0
    prob = opstd.Problem(shape, bcs, dx, dt, c0)
    rng = np.random.default_rng(sum(shape) + 1)
    p = prob.project(rng.standard_normal(shape))
    a = [i for i in range(len(shape)) if bcs[i][0] == P][0]
    u = rng.standard_normal(prob.u_shape(a))
    refs = (-(dt / prob.rho0) * prob.grad(p, a), -(dt * prob.rho0 * c0 ** 2) * prob.div(u, a))
    paths = ("fft", "per_axis") if shape[a] <= 4096 else ("fft",)
    got = {}
    for path in paths:
        with Plan(shape, dx, dt, c0, bcs, precision="fp32") as plan:
            plan.set_path(path)
            st = plan.new_state(p)
            for b in range(len(shape)):
                st.u[b].zero_()
            plan.apply_axis(st, a, 0)
            torch.cuda.synchronize()
            got[(path, 0)] = st.u[a].double().cpu().numpy()
            st = plan.new_state(np.zeros(shape))
            st.u[a].copy_(torch.from_numpy(u).to(st.u[a].dtype))
            plan.apply_axis(st, a, 1)
            torch.cuda.synchronize()
            got[(path, 1)] = st.p.double().cpu().numpy()
    for which in (0, 1):
        e = rel_l2(got[("fft", which)], refs[which])
        print("axis", a, "which", which, "rel_l2", e, flush=True)
        assert e < 2e-6
        if "per_axis" in paths:
            assert rel_l2(got[("per_axis", which)], refs[which]) < 2e-6
            assert not np.array_equal(got[("fft", which)], got[("per_axis", which)])


@pytest.mark.parametrize("shape,bcs,steps", [((512, 96), ((P, P), (N, D)), 60),
                                             ((64, 48, 256), ((D, N), (N, N), (P, P)), 30)])
def test_pow2_kernel_periodic_steps(shape, bcs, steps):
    # full steps with a periodic axis on the FFT path and wall-bounded axes on the dense path, against the
    # oracle's run of the same steps
    import workloads
    from gpu_helpers import oracle_problem, run_gpu

    print("case", shape, bcs, steps, flush=True)
    dx, c0 = 1e-3, 1500.0
    dt = (0.25 if len(shape) == 2 else 0.2) * dx / c0
    centre = tuple(s * dx / 2.2 for s in shape)
    p0 = workloads.gaussian(shape, dx, centre, 5 * dx)
    case = workloads.Case("pow2_periodic", shape, bcs, dx, dt, c0, steps, p0)
    ref_p, ref_u = oracle_problem(case).run(p0, steps)
    got_p, got_u = run_gpu(case, precision="fp32", path="fft")
    e = rel_l2(got_p, ref_p)
    print("rel_l2 p", e, "u", [rel_l2(g, r) for g, r in zip(got_u, ref_u)], flush=True)
    assert e < 1e-5
    for g, r in zip(got_u, ref_u):
        assert rel_l2(g, r) < 1e-5


MULTI_CASES = [
    ((129, 129), ((D, N), (N, D)), False, 40),
    ((257, 257), ((N, N), (D, D)), True, 40),
    ((256, 256), ((P, P), (P, P)), False, 40),
    ((129, 129, 129), ((D, D), (N, D), (N, N)), False, 8),
    ((256, 256, 256), ((P, P), (P, P), (P, P)), False, 4),
]


@pytest.mark.parametrize("shape,bcs,medium,steps", MULTI_CASES)
def test_pow2_velocity_axes_in_one_launch(shape, bcs, medium, steps):
    # when every axis runs on the power-of-two kernel with one transform length, a step launches the
    # velocity terms of all axes together; compare one step with the same terms launched axis by axis,
    # and a few steps with the oracle
    import torch
    import workloads
    from gpu_helpers import oracle_problem, run_gpu
    from paper_2005_00322_amd import Plan

    print("case", shape, bcs, "c0 map" if medium else "", steps, flush=True)
    dx = 1e-3
    rng = np.random.default_rng(sum(shape) + 7)
    c0_map = workloads.smooth_c0_map(rng, shape) if medium else None
    c0 = float(c0_map.max()) if medium else 1500.0
    dt = (0.25 if len(shape) == 2 else 0.2) * dx / c0
    centre = tuple(s * dx / 2.2 for s in shape)
    p0 = workloads.gaussian(shape, dx, centre, 5 * dx)
    prob = opstd.Problem(shape, bcs, dx, dt, c0)
    p = prob.project(p0 + 0.1 * rng.standard_normal(shape))
    us = [rng.standard_normal(prob.u_shape(a)) for a in range(len(shape))]
    out = []
    with Plan(shape, dx, dt, c0, bcs, precision="fp32", c0_map=c0_map) as plan:
        plan.set_path("fft")
        for merged in (True, False):
            st = plan.new_state(p)
            for a in range(len(shape)):
                st.u[a].copy_(torch.from_numpy(us[a]).to(st.u[a].dtype))
            if merged:
                plan.step(st, 1)
            else:
                for which in (0, 1):
                    for a in range(len(shape)):
                        plan.apply_axis(st, a, which)
            torch.cuda.synchronize()
            out.append([st.p.double().cpu().numpy()] + [u.double().cpu().numpy() for u in st.u])
    for x, y in zip(*out):
        d = np.max(np.abs(x - y))
        print("max |merged - per axis|", d, "bitwise" if d == 0 else "", flush=True)
        assert d <= 1e-6 * np.max(np.abs(y))
    case = workloads.Case("pow2_multi", shape, bcs, dx, dt, c0, steps, p0, c0_map=c0_map)
    ref = workloads.Case("pow2_multi", shape, bcs, dx, dt, c0, steps, p0,
                         c0_map=None if c0_map is None else c0_map.astype(np.float32).astype(np.float64))
    ref_p, ref_u = oracle_problem(ref).run(p0, steps)
    got_p, got_u = run_gpu(case, precision="fp32", path="fft")
    e = rel_l2(got_p, ref_p)
    print("rel_l2 p", e, "u", [rel_l2(g, r) for g, r in zip(got_u, ref_u)], flush=True)
    assert e < 1e-5
    for g, r in zip(got_u, ref_u):
        assert rel_l2(g, r) < 1e-5


def test_pow2_velocity_launch_graph_chunks_bitwise():
    # the two-axis velocity launch inside captured step graphs of several lengths gives bitwise the
    # result of one long run
    import workloads
    from gpu_helpers import run_gpu

    shape, bcs = (257, 257), ((D, N), (N, D))
    dx, c0 = 1e-3, 1500.0
    p0 = workloads.gaussian(shape, dx, (100 * dx, 140 * dx), 6 * dx)
    case = workloads.Case("pow2_multi_chunks", shape, bcs, dx, 0.25 * dx / c0, c0, 120, p0)
    print("case", shape, bcs, flush=True)
    p1, u1 = run_gpu(case, "fp32", path="fft")
    p2, u2 = run_gpu(case, "fp32", path="fft", chunks=[50, 3, 67])
    assert np.array_equal(p1, p2)
    for a, b in zip(u1, u2):
        assert np.array_equal(a, b)
