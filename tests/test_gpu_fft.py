"""GPU parity of the FFT path (axes applied as LDS-resident FFTs of the symmetric extension).

Small shapes force the FFT path on every axis and compare with the FP64 oracle element by element;
large shapes run it where the automatic choice takes it (axes above 512 nodes) and compare with the
oracle's closed forms (the modal solution at 2049^2; a single basis function per axis at 1025^3, on
sampled points).  Tolerances as elsewhere: FP64 1e-10, FP32 1e-5, split-bf16 plans 1e-3.
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import TOL, oracle_problem, rel_l2, run_gpu
from oracle import pstd as opstd

pytestmark = pytest.mark.gpu
N, D = opstd.NEUMANN, opstd.DIRICHLET


def _print(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("seed,ndim", [(0, 1), (1, 2), (2, 2), (3, 3), (4, 3), (5, 2)])
def test_single_operator_application(prec, seed, ndim):
    # one velocity and one pressure term per axis: the FFT operator against the oracle's DTT recipe
    import torch
    from paper_2005_00322_amd import Plan

    case = workloads.fft_small_case(seed, ndim)
    _print("case", case.name, case.shape, case.bcs, prec)
    prob = oracle_problem(case)
    rng = np.random.default_rng(77 + seed)
    p = prob.project(rng.standard_normal(case.shape))
    us = [rng.standard_normal(prob.u_shape(a)) for a in range(ndim)]
    tol = 1e-13 if prec == "fp64" else 2e-6
    with Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, precision=prec) as plan:
        plan.set_path("fft")
        for a in range(ndim):
            st = plan.new_state(p)
            for b in range(ndim):
                st.u[b].zero_()
            plan.apply_axis(st, a, 0)
            torch.cuda.synchronize()
            ref = -(case.dt / case.rho0) * prob.grad(p, a)
            assert rel_l2(st.u[a].double().cpu().numpy(), ref) < tol
            st = plan.new_state(np.zeros(case.shape))
            st.u[a].copy_(torch.from_numpy(us[a]).to(st.u[a].dtype))
            plan.apply_axis(st, a, 1)
            torch.cuda.synchronize()
            ref = -(case.dt * case.rho0 * case.c0 ** 2) * prob.div(us[a], a)
            assert rel_l2(st.p.double().cpu().numpy(), ref) < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_bf16"])
@pytest.mark.parametrize("seed,ndim", [(10, 1), (11, 2), (12, 2), (13, 3), (14, 3), (15, 2), (16, 3)])
def test_steps_forced_fft(prec, seed, ndim):
    case = workloads.fft_small_case(seed, ndim, steps=40)
    _print("case", case.name, case.shape, case.bcs, prec)
    p, u = run_gpu(case, prec, path="fft")
    po, uo = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL[prec]
    for a in range(ndim):
        assert rel_l2(u[a], uo[a]) < TOL[prec]


def test_graph_chunks_bitwise_fft():
    case = workloads.fft_small_case(21, 2, steps=120)
    _print("case", case.name, case.shape)
    p1, _ = run_gpu(case, "fp32", path="fft")
    p2, _ = run_gpu(case, "fp32", path="fft", chunks=[50, 3, 67])
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("shape,bcs", [((513, 97), ((D, N), (N, D))), ((769, 65), ((N, N), (D, D))),
                                       ((97, 641), ((D, D), (N, D))), ((1025, 40), ((N, D), (D, N)))])
def test_auto_path_large_axis_vs_oracle(shape, bcs):
    # axes above 512 nodes take the FFT path automatically; the others stay dense
    rng = np.random.default_rng(sum(shape))
    c0, dx = 1500.0, 1e-4
    p0 = workloads.gaussian(shape, dx, tuple(s * dx / 2.3 for s in shape), 6 * dx)
    p0 += 0.05 * rng.standard_normal(shape)
    case = workloads.Case("auto_%dx%d" % shape, shape, bcs, dx, 0.3 * dx / c0, c0, 60, p0)
    _print("case", case.name, bcs)
    p, _ = run_gpu(case, "fp32")
    po, _ = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL["fp32"]
    # same step on the dense path (both on the GPU)
    pd, _ = run_gpu(case, "fp32", path="per_axis")
    assert rel_l2(p, pd) < TOL["fp32"]


def test_fft_with_sound_speed_map():
    shape = (129, 97)
    bcs = ((D, N), (N, N))
    rng = np.random.default_rng(5)
    c0_map = workloads.smooth_c0_map(rng, shape)
    dx = 1e-4
    dt = 0.25 * dx / float(c0_map.max())
    p0 = workloads.gaussian(shape, dx, (60 * dx, 40 * dx), 5 * dx)
    case = workloads.Case("map_fft", shape, bcs, dx, dt, float(c0_map.max()), 50, p0, c0_map=c0_map)
    p, _ = run_gpu(case, "fp32", path="fft")
    # the device sees the float32 map
    case32 = workloads.Case("map_fft", shape, bcs, dx, dt, case.c0, 50, p0,
                            c0_map=c0_map.astype(np.float32).astype(np.float64))
    po, _ = oracle_problem(case32).run(p0, 50)
    assert rel_l2(p, po) < TOL["fp32"]


@pytest.mark.parametrize("prec,n", [("fp64", 2049), ("fp32", 2049), ("fp32", 4097), ("fp64", 4097), ("fp32", 8193)])
def test_1d_long_axis(prec, n):
    # 1D plans above 1365 nodes run on the FFT path; 4097 (FP64) and 8193 (FP32) are the largest a plan
    # takes there (transforms of 8192 and 16384 points, one per block in more than 64 KB of LDS)
    dx, c0 = 1e-4, 1500.0
    bcs = ((N, D),)
    p0 = workloads.gaussian((n,), dx, (0.37 * n * dx,), 8 * dx)
    case = workloads.Case("long1d", (n,), bcs, dx, 0.4 * dx / c0, c0, 300, p0, precision=prec)
    _print("case 1d", n, prec)
    p, _ = run_gpu(case, prec)
    prob = oracle_problem(case)
    ref = prob.modal_solution(p0, case.steps)
    assert rel_l2(p, ref) < TOL[prec]


def test_2d_2049_workload_vs_modal_closed_form():
    case = workloads.pstd2d_large()
    _print("case", case.name, case.steps)
    p, _ = run_gpu(case, "fp32")
    ref = oracle_problem(case).modal_solution(case.p0, case.steps)
    err = rel_l2(p, ref)
    _print("pstd2d_large rel L2", err)
    assert err < TOL["fp32"]


def test_3d_1025_single_mode_sampled():
    # one basis function per axis evolves as cos(m theta) p0 (sampled comparison at 1025^3)
    import torch
    from paper_2005_00322_amd import Plan

    case = workloads.pstd3d_mode()
    n = case.shape[0]
    fs, ksq = [], 0.0
    for a, m in enumerate(case.extra["modes"]):
        f, k = opstd.axis_mode(n, case.bcs[a][0], case.bcs[a][1], case.dx, m)
        fs.append(f)
        ksq += k * k
    th = opstd.mode_phase(case.c0, case.dt, ksq)
    _print("case", case.name, case.bcs, case.extra["modes"])
    dev = torch.device("cuda")
    fx, fy, fz = (torch.from_numpy(f.astype(np.float32)).to(dev) for f in fs)
    with Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, precision="fp32") as plan:
        st = plan.new_state(None)
        st.p.copy_(fx[:, None, None] * fy[None, :, None] * fz[None, None, :])
        plan.init_state(st)
        plan.step(st, case.steps)
        torch.cuda.synchronize()
        rng = np.random.default_rng(3)
        idx = rng.integers(0, n, size=(200000, 3))
        t_idx = torch.from_numpy(idx).to(dev)
        got = st.p[t_idx[:, 0], t_idx[:, 1], t_idx[:, 2]].double().cpu().numpy()
    ref = np.cos(case.steps * th) * fs[0][idx[:, 0]] * fs[1][idx[:, 1]] * fs[2][idx[:, 2]]
    err = rel_l2(got, ref)
    _print("pstd3d_mode sampled rel L2", err, "phase", case.steps * th)
    assert err < TOL["fp32"]
