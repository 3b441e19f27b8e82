"""Shared helpers of the GPU tests: run a workload case through the C ABI and through the oracle."""
import numpy as np

from oracle import pstd as opstd

TOL = {"fp64": 1e-10, "fp32": 1e-5, "split_bf16": 1e-3}


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_problem(case):
    return opstd.Problem(case.shape, case.bcs, case.dx, case.dt, case.c0, rho0=case.rho0, c0_map=case.c0_map)


def run_gpu(case, precision=None, steps=None, u_mode="centred", chunks=None, path=None):
    """Returns (p, [u_a]) as float64 numpy arrays after stepping on the GPU."""
    import torch
    from paper_2005_00322_amd import Plan

    precision = precision or case.precision
    steps = case.steps if steps is None else steps
    c0 = case.c0 if case.c0_map is None else float(np.max(case.c0_map))
    with Plan(case.shape, case.dx, case.dt, c0, case.bcs, rho0=case.rho0, precision=precision,
              c0_map=case.c0_map) as plan:
        if path is not None:
            plan.set_path(path)
        st = plan.new_state(case.p0)
        plan.init_state(st, u_mode)
        for n in (chunks or [steps]):
            plan.step(st, n)
        torch.cuda.synchronize()
        return st.p.double().cpu().numpy(), [u.double().cpu().numpy() for u in st.u]
