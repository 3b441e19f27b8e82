"""GPU parity of the split-bf16 contractions that form their operator slices on the chip from the
operators' Toeplitz and Hankel parts (axes whose operators have 193..384 rows): against the FP64 oracle,
and against the same plan reading its stored operators (path "stored").  The cases cover every boundary
family, half-width tail tiles, a c0(x) map and the three field layouts (strided with one and with many
outer blocks, contiguous rows with and without 16-byte alignment)."""
import numpy as np
import pytest

import workloads
from gpu_helpers import TOL, oracle_problem, rel_l2, run_gpu
from oracle import pstd as opstd

pytestmark = pytest.mark.gpu
N, D, P = opstd.NEUMANN, opstd.DIRICHLET, workloads.PERIODIC
NH, DH = workloads.NEUMANN_HALF, workloads.DIRICHLET_HALF

CASES = [
    (1, (300, 260), ((N, D), (D, N)), 60),
    (2, (257, 385), ((N, N), (D, D)), 60),
    (3, (230, 250), ((N, DH), (D, NH)), 60),
    (4, (240, 300), ((P, P), (D, N)), 60),
    (5, (200, 232, 216), ((D, N), (D, D), (N, D)), 25),
    (6, (196, 201, 385), ((N, N), (N, D), (D, D)), 12),
]


def _case(seed, shape, bcs, steps, c0_map=False):
    rng = workloads.rng_for(9000 + seed)
    dx, c0 = 1e-4, float(rng.uniform(1400, 1600))
    centre = [rng.uniform(0.3, 0.7) * (n - 1) * dx for n in shape]
    p0 = workloads.gaussian(shape, dx, centre, 6 * dx)
    cmap = workloads.smooth_c0_map(rng, shape) if c0_map else None
    cmax = c0 if cmap is None else float(cmap.max())
    return workloads.Case("structured", shape, bcs, dx, 0.3 * dx / cmax, c0, steps, p0, precision="split_bf16",
                          c0_map=cmap)


@pytest.mark.parametrize("seed,shape,bcs,steps", CASES)
def test_formed_operators_match_oracle(seed, shape, bcs, steps):
    case = _case(seed, shape, bcs, steps)
    print("structured", shape, bcs, steps, flush=True)
    p, u = run_gpu(case, "split_bf16")
    ps, us = run_gpu(case, "split_bf16", path="stored")
    ref = oracle_problem(case).modal_solution(case.p0, steps)
    assert rel_l2(p, ref) < TOL["split_bf16"]
    assert rel_l2(ps, ref) < TOL["split_bf16"]
    # the two paths round the operators differently (FP32 sum of the parts against the FP64 entry)
    assert not np.array_equal(p, ps)
    assert rel_l2(p, ps) < TOL["split_bf16"]
    for a in range(len(shape)):
        assert rel_l2(u[a], us[a]) < TOL["split_bf16"]


def test_formed_operators_with_c0_map():
    case = _case(7, (280, 210), ((D, N), (N, D)), 40, c0_map=True)
    print("structured c0 map", case.shape, flush=True)
    p, _ = run_gpu(case, "split_bf16")
    po, _ = oracle_problem(case).run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL["split_bf16"]
