"""GPU parity of the collocated derivatives (§3.3) and half-step interpolations (§3.4) applied along an
axis of a device field (pstd_apply_axis_operator) against the oracle's operators, in FP64, FP32 and
split-bf16, on 1D/2D/3D grids with ragged tiles, and sampled lines at 384^3."""
import numpy as np
import pytest

from gpu_helpers import TOL, rel_l2
from oracle import pstd as o

pytestmark = pytest.mark.gpu
N, D = o.NEUMANN, o.DIRICHLET
KINDS = (2, 3, 4, 5)


def _in_extent(n, which):
    return n if which in (2, 4) else n - 1


def _oracle_apply(x, axis, ax, which):
    A = ax.resample_matrix(which)
    return np.moveaxis(np.tensordot(A, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)


def _run(shape, bcs, prec, seed):
    import torch

    from paper_2005_00322_amd import Plan
    rng = np.random.default_rng(seed)
    dx = 1e-4
    with Plan(shape, dx, 1e-8, 1500.0, bcs, precision=prec) as plan:
        for axis in range(len(shape)):
            ax = o.Axis(shape[axis], bcs[axis][0], bcs[axis][1], dx)
            for which in KINDS:
                s = list(shape)
                s[axis] = _in_extent(shape[axis], which)
                x = rng.standard_normal(s)
                xt = torch.as_tensor(x, dtype=plan.dtype, device="cuda").contiguous()
                print("resample", shape, bcs, prec, axis, which, flush=True)
                got = plan.apply_operator(axis, which, xt)
                torch.cuda.synchronize()
                want = _oracle_apply(x, axis, ax, which)
                assert got.shape == want.shape
                assert rel_l2(got.double().cpu().numpy(), want) < TOL[prec], (axis, which)


GRIDS = [
    (1, (17,), ((N, D),)),
    (2, (130,), ((D, D),)),
    (3, (600,), ((N, N),)),
    (4, (36, 28), ((N, N), (D, N))),
    (5, (300, 70), ((D, N), (N, D))),
    (6, (14, 18, 16), ((D, D), (N, N), (N, D))),
    (7, (9, 33, 65), ((N, D), (D, N), (D, D))),
    (8, (3, 3), ((D, D), (N, D))),                       # minimal axes
    (9, (3,), ((N, N),)),
]


# (a 1D split-bf16 plan computes as FP32)
@pytest.mark.parametrize("prec,seed,shape,bcs", [(p,) + g for p in ("fp64", "fp32", "split_bf16") for g in GRIDS])
def test_parity(prec, seed, shape, bcs):
    _run(shape, bcs, prec, seed)


def test_velocity_on_nodes_after_steps():
    """u resampled onto the p nodes after 50 steps equals the oracle's interpolation of its own u."""
    import torch

    import workloads
    from gpu_helpers import oracle_problem, run_gpu
    from paper_2005_00322_amd import STAG_TO_NODES, Plan
    case = workloads.pstd2d(scale=0.25, steps=50)
    prob = oracle_problem(case)
    _, uo = prob.run(case.p0, case.steps)
    with Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, precision="fp32") as plan:
        st = plan.new_state(case.p0)
        plan.init_state(st)
        plan.step(st, case.steps)
        for a in range(2):
            got = plan.apply_operator(a, STAG_TO_NODES, st.u[a])
            torch.cuda.synchronize()
            ax = o.Axis(case.shape[a], case.bcs[a][0], case.bcs[a][1], case.dx)
            want = _oracle_apply(uo[a], a, ax, STAG_TO_NODES)
            assert rel_l2(got.double().cpu().numpy(), want) < TOL["fp32"]


def test_full_size_sampled_lines():
    """384^3 split-bf16 (the 3D workload's plan): every operator along every axis, checked on 24 sampled
    lines against the oracle's matrix applied to the same lines."""
    import torch

    import workloads
    from paper_2005_00322_amd import Plan
    case = workloads.pstd3d()
    rng = np.random.default_rng(11)
    n = case.shape
    with Plan(case.shape, case.dx, case.dt, case.c0, case.bcs, precision="split_bf16") as plan:
        for axis in range(3):
            ax = o.Axis(n[axis], case.bcs[axis][0], case.bcs[axis][1], case.dx)
            for which in (3, 5):
                A = ax.resample_matrix(which)
                s = list(n)
                s[axis] = A.shape[1]
                x = torch.randn(s, device="cuda", dtype=torch.float32)
                print("resample 384^3", axis, which, flush=True)
                y = plan.apply_operator(axis, which, x)
                torch.cuda.synchronize()
                xm = torch.movedim(x, axis, -1)
                ym = torch.movedim(y, axis, -1)
                for _ in range(24):
                    i, j = (int(v) for v in rng.integers(0, [xm.shape[0], xm.shape[1]]))
                    line = xm[i, j].double().cpu().numpy()
                    assert rel_l2(ym[i, j].double().cpu().numpy(), A @ line) < TOL["split_bf16"]


def test_argument_errors():
    import torch

    from paper_2005_00322_amd import PERIODIC, Plan, PstdError
    with Plan((16, 20), 1e-4, 1e-8, 1500.0, ((PERIODIC, PERIODIC), (N, D)), precision="fp32") as plan:
        x = torch.zeros((16, 20), device="cuda")
        with pytest.raises(PstdError):
            plan.apply_operator(0, 2, x)            # periodic axis
        with pytest.raises(ValueError):
            plan.apply_operator(1, 2, torch.zeros((16, 19), device="cuda"))
