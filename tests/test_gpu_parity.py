"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded inputs.

Tolerances (relative L2 over the whole field): FP32 1e-5 and split-bf16 1e-3 (the stated targets);
FP64 1e-10 (rounding of ~2n-term dot products accumulated over the step count, far below it).
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import TOL, oracle_problem, rel_l2, run_gpu
from oracle import images
from oracle import pstd as opstd

pytestmark = pytest.mark.gpu
N, D = opstd.NEUMANN, opstd.DIRICHLET


def _print_case(case, prec):
    print("case", case.name, case.shape, case.bcs, prec, "steps", case.steps, flush=True)


def test_1d_workload_fp64():
    case = workloads.pstd1d()
    _print_case(case, "fp64")
    p, u = run_gpu(case, "fp64")
    prob = oracle_problem(case)
    po, uo = prob.run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL["fp64"]
    assert rel_l2(u[0], uo[0]) < TOL["fp64"]
    assert rel_l2(p, prob.modal_solution(case.p0, case.steps)) < TOL["fp64"]


def test_1d_workload_fp32():
    case = workloads.pstd1d(precision="fp32")
    _print_case(case, "fp32")
    p, _ = run_gpu(case, "fp32")
    po, _ = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL["fp32"]


def test_1d_image_source_fp64():
    # Dirichlet/Neumann box, image-summed Gaussian: GPU vs the transform-free image solution
    n, dx, c0 = 97, 1e-4, 1500.0
    dt = 0.3 * dx / c0
    bcs = ((D, N),)
    centre, sigma = (30 * dx,), 4 * dx
    p0 = images.image_summed_gaussian((n,), bcs, dx, centre, 1.0, sigma)
    case = workloads.Case("img1d", (n,), bcs, dx, dt, c0, 700, p0, precision="fp64")
    p, _ = run_gpu(case)
    ref = images.image_solution((n,), bcs, dx, c0, dt, 700, centre, 1.0, sigma)
    assert rel_l2(p, ref) < 1e-9


@pytest.mark.parametrize("prec,n,path", [("fp64", 1400, None), ("fp32", 1400, None), ("fp64", 2049, "per_axis"),
                                         ("fp32", 2049, "per_axis")])
def test_1d_walls_above_single_workgroup(prec, n, path):
    # walls on nodes above 1365 nodes: 2(n-1) = 2798 has the prime factor 1399, so the 1400-node axis runs
    # on the dense contraction path; the 2049-node axis is moved there from the FFT path
    dx, c0 = 1e-4, 1500.0
    bcs = ((D, N),)
    p0 = workloads.gaussian((n,), dx, (0.37 * (n - 1) * dx,), 8 * dx)
    case = workloads.Case("walls1d", (n,), bcs, dx, 0.4 * dx / c0, c0, 120, p0, precision=prec)
    _print_case(case, prec)
    p, _ = run_gpu(case, prec, path=path)
    ref = oracle_problem(case).modal_solution(p0, case.steps)
    assert rel_l2(p, ref) < TOL[prec]


@pytest.mark.parametrize("steps", [1, 7, 49, 50, 57, 120])
def test_any_step_count_replays_graphs(steps):
    # every step count replays captured graphs (whole chunks of 50 steps, then one of the rest); the
    # result equals single steps and the oracle
    case = workloads.random_small_case(21, 3, max_n=20, steps=steps)
    _print_case(case, "fp32")
    p1, _ = run_gpu(case, "fp32")
    p2, _ = run_gpu(case, "fp32", chunks=[1] * steps)
    po, _ = oracle_problem(case).run(case.p0, steps)
    assert np.array_equal(p1, p2)
    assert rel_l2(p1, po) < TOL["fp32"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_bf16"])
@pytest.mark.parametrize("seed,ndim", [(10, 2), (11, 2), (12, 3), (13, 3), (14, 2)])
def test_random_small(prec, seed, ndim):
    case = workloads.random_small_case(seed, ndim, max_n=40 if ndim == 2 else 24, steps=40)
    _print_case(case, prec)
    p, u = run_gpu(case, prec)
    po, uo = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL[prec]
    for a in range(ndim):
        assert rel_l2(u[a], uo[a]) < TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_bf16"])
@pytest.mark.parametrize("shape,bcs", [
    ((150, 133), ((D, N), (N, D))),            # several tiles and a ragged tail on both axes
    ((257, 129), ((N, N), (D, D))),
    ((70, 45, 37), ((D, D), (N, D), (N, N))),
    ((33, 140, 67), ((N, D), (D, N), (D, D))),
])
def test_multi_tile_shapes(prec, shape, bcs):
    rng = np.random.default_rng(sum(shape))
    c0 = 1500.0
    dt = (0.25 if len(shape) == 3 else 0.3) * 1e-4 / c0
    case = workloads.Case("tiles", shape, bcs, 1e-4, dt, c0, 30, rng.standard_normal(shape), precision=prec)
    _print_case(case, prec)
    p, u = run_gpu(case, prec)
    po, uo = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL[prec]
    for a in range(len(shape)):
        assert rel_l2(u[a], uo[a]) < TOL[prec]


@pytest.mark.parametrize("u_mode", ["centred", "zero"])
def test_state_init(u_mode):
    case = workloads.random_small_case(21, 3, max_n=30, steps=0)
    p, u = run_gpu(case, "fp64", steps=0, u_mode=u_mode)
    prob = oracle_problem(case)
    assert np.max(np.abs(p - prob.project(case.p0))) == 0.0       # Dirichlet nodes zeroed exactly
    uo = prob.initial_velocity(case.p0, u_mode)
    for a in range(3):
        if u_mode == "zero":
            assert np.all(u[a] == 0.0)
        else:
            assert rel_l2(u[a], uo[a]) < 1e-12


def test_sound_speed_map_2d():
    rng = np.random.default_rng(5)
    shape = (60, 75)
    # the device receives the map as float32; the oracle gets the same values
    cmap = workloads.smooth_c0_map(rng, shape).astype(np.float32).astype(np.float64)
    dt = 0.3 * 1e-4 / 1600.0
    case = workloads.Case("map2d", shape, ((D, D), (N, N)), 1e-4, dt, 1500.0, 120,
                          workloads.gaussian(shape, 1e-4, (30e-4, 40e-4), 4e-4), c0_map=cmap)
    for prec in ("fp64", "fp32"):
        p, _ = run_gpu(case, prec)
        po, _ = oracle_problem(case).run(case.p0, case.steps)
        assert rel_l2(p, po) < TOL[prec]


@pytest.mark.parametrize("path", ["per_axis", "fused"])
@pytest.mark.parametrize("shape,bcs", [
    ((3, 3), ((N, N), (D, N))),                 # smallest grid
    ((150, 133), ((D, N), (N, D))),
    ((37, 500), ((D, D), (N, N))),
    ((512, 512), ((N, D), (D, D))),             # largest grid of the fused path
    ((129, 257), ((N, D), (D, N))),             # last tile rows past the allocated operator rows
])
def test_2d_paths_fp32(path, shape, bcs):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    c0 = 1500.0
    case = workloads.Case("paths", shape, bcs, 1e-4, 0.3e-4 / c0, c0, 25, rng.standard_normal(shape))
    _print_case(case, "fp32 " + path)
    p, u = run_gpu(case, "fp32", path=path)
    po, uo = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL["fp32"]
    for a in range(2):
        assert rel_l2(u[a], uo[a]) < TOL["fp32"]


def test_2d_fused_with_map():
    rng = np.random.default_rng(9)
    shape = (97, 130)
    cmap = workloads.smooth_c0_map(rng, shape).astype(np.float32).astype(np.float64)
    case = workloads.Case("pmap", shape, ((N, D), (D, N)), 1e-4, 0.3e-4 / 1600.0, 1500.0, 150,
                          workloads.gaussian(shape, 1e-4, (50e-4, 60e-4), 4e-4), c0_map=cmap)
    p, _ = run_gpu(case, "fp32", path="fused")
    po, _ = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL["fp32"]


@pytest.mark.parametrize("path", ["per_axis", "fused"])
def test_graph_chunks_equal_single_steps(path):
    # the same kernels in the same order, whether replayed from graphs, launched directly or run
    # fusedly in one launch per call: bitwise equal results (also the resume-from-checkpoint case)
    case = workloads.random_small_case(30, 2, max_n=40, steps=137)
    a, ua = run_gpu(case, "fp32", chunks=[137], path=path)
    b, ub = run_gpu(case, "fp32", chunks=[1] * 37 + [100], path=path)
    assert np.array_equal(a, b)
    for x, y in zip(ua, ub):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("path", ["per_axis", "fused"])
def test_2d_workload_full_fp32(path):
    case = workloads.pstd2d()
    _print_case(case, "fp32 " + path)
    p, _ = run_gpu(case, "fp32", path=path)
    prob = oracle_problem(case)
    ref = prob.modal_solution(case.p0, case.steps)
    err = rel_l2(p, ref)
    print("2d fp32", path, "rel L2", err, flush=True)
    assert err < TOL["fp32"]


def test_3d_workload_full_split_bf16():
    case = workloads.pstd3d()
    _print_case(case, "split_bf16")
    p, _ = run_gpu(case, "split_bf16")
    ref = oracle_problem(case).modal_solution(case.p0, case.steps)
    err = rel_l2(p, ref)
    print("3d split-bf16 rel L2", err, flush=True)
    assert err < TOL["split_bf16"]


def test_operators_roundtrip():
    import torch
    from paper_2005_00322_amd import Plan
    shape, bcs, dx, c0 = (40, 33), ((N, D), (D, D)), 1e-4, 1500.0
    dt = 0.3 * dx / c0
    prob = opstd.Problem(shape, bcs, dx, dt, c0)
    for prec, tol in (("fp64", 1e-15), ("fp32", 1e-7), ("split_bf16", 2e-5)):
        with Plan(shape, dx, dt, c0, bcs, precision=prec) as plan:
            for a in range(2):
                G = plan.operator(a, 0)
                Dm = plan.operator(a, 1)
                Gr = -(dt / 1000.0) * prob.axes[a].grad_matrix()
                Dr = -(dt * 1000.0 * c0 ** 2) * prob.axes[a].div_matrix()
                assert np.max(np.abs(G - Gr)) <= tol * np.max(np.abs(Gr))
                assert np.max(np.abs(Dm - Dr)) <= tol * np.max(np.abs(Dr))
    torch.cuda.synchronize()


def test_check_finite_flags_planted_nan():
    import torch
    from paper_2005_00322_amd import Plan
    shape = (20, 30)
    with Plan(shape, 1e-4, 1e-8, 1500.0, ((N, N), (N, N))) as plan:
        st = plan.new_state(np.ones(shape))
        plan.init_state(st)
        assert plan.check_finite(st)
        st.u[1][3, 4] = float("nan")
        assert not plan.check_finite(st)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec,shape,bcs", [
    ("fp32", (41, 36, 37), ((N, D), (D, D), (D, N))),
    ("split_bf16", (41, 36, 37), ((N, D), (D, D), (D, N))),
    ("fp32", (65, 46), ((D, N), (N, D))),        # 2D: the fused phase kernels
])
def test_misaligned_state_buffers(prec, shape, bcs):
    # state tensors that start 4 bytes past a 16-byte boundary take the scalar-load paths
    import torch
    from paper_2005_00322_amd import Plan, State
    rng = np.random.default_rng(77)
    p0 = rng.standard_normal(shape)
    c0 = 1500.0
    dt = 0.25e-4 / c0
    case = workloads.Case("misaligned", shape, bcs, 1e-4, dt, c0, 20, p0, precision=prec)

    def offset_view(sh, init=None):
        n = int(np.prod(sh))
        buf = torch.zeros(n + 1, dtype=torch.float32, device="cuda")
        v = buf[1:].view(sh)
        if init is not None:
            v.copy_(torch.as_tensor(init, dtype=torch.float32))
        assert v.data_ptr() % 16 == 4
        return buf, v

    with Plan(shape, 1e-4, dt, c0, bcs, precision=prec) as plan:
        keep = []
        bp, p = offset_view(shape, p0)
        keep.append(bp)
        us = []
        for a in range(len(shape)):
            bu, u = offset_view(plan.u_shape(a))
            keep.append(bu)
            us.append(u)
        st = State(p, us, 0)
        plan.init_state(st)
        plan.step(st, case.steps)
        torch.cuda.synchronize()
        got = p.double().cpu().numpy()
    po, _ = oracle_problem(case).run(p0, case.steps)
    assert rel_l2(got, po) < TOL[prec]
