"""GPU parity of axes whose right wall lies half a step beyond the last node (groups III/IV, DTT types
V-VIII) against the FP64 oracle: 1D/2D/3D mixed with other walls and periodic axes in FP64, FP32 and
split-bf16, both 2D FP32 paths, and a reflected pulse equal to its image sources."""
import numpy as np
import pytest

import workloads
from gpu_helpers import TOL, oracle_problem, rel_l2, run_gpu
from oracle import images
from oracle import pstd as opstd

pytestmark = pytest.mark.gpu
N, D, P = opstd.NEUMANN, opstd.DIRICHLET, opstd.PERIODIC
NH, DH = opstd.NEUMANN_HALF, opstd.DIRICHLET_HALF


def _case(seed, shape, bcs, steps, precision):
    rng = np.random.default_rng(seed)
    dx, c0 = 1e-4, float(rng.uniform(1400, 1600))
    dt = 0.3 * dx / c0
    p0 = rng.standard_normal(shape)
    return workloads.Case("halfwall_%d" % seed, shape, bcs, dx, dt, c0, steps, p0, precision=precision)


def _check(case, path=None):
    p, u = run_gpu(case, path=path)
    prob = oracle_problem(case)
    po, uo = prob.run(case.p0, case.steps)
    assert rel_l2(p, po) < TOL[case.precision]
    for a in range(len(case.shape)):
        assert u[a].shape == prob.u_shape(a)
        assert rel_l2(u[a], uo[a]) < TOL[case.precision]


GRIDS = [
    (1, (40,), ((N, NH),)),
    (2, (129,), ((D, DH),)),
    (3, (36, 28), ((N, DH), (D, N))),
    (4, (30, 41), ((D, D), (D, NH))),
    (5, (24, 20), ((N, NH), (P, P))),
    (6, (14, 18, 16), ((D, NH), (N, DH), (N, D))),
    (7, (12, 10, 17), ((N, N), (P, P), (D, DH))),
]


@pytest.mark.parametrize("prec,seed,shape,bcs", [(p,) + g for p in ("fp64", "fp32", "split_bf16") for g in GRIDS
                                                 if not (p == "split_bf16" and len(g[1]) == 1)])
def test_parity(prec, seed, shape, bcs):
    print("halfwall", shape, bcs, prec, flush=True)
    _check(_case(seed, shape, bcs, 40, prec))


@pytest.mark.parametrize("path", ["fused", "per_axis"])
@pytest.mark.parametrize("seed,shape,bcs", [
    (11, (36, 28), ((N, NH), (N, DH))),
    (12, (300, 70), ((D, DH), (N, D))),      # the 512-wide instance, ragged tiles
    (13, (17, 259), ((P, P), (D, NH))),
])
def test_2d_fp32_paths(path, seed, shape, bcs):
    print("halfwall 2d", path, shape, bcs, flush=True)
    _check(_case(seed, shape, bcs, 60, "fp32"), path=path)


@pytest.mark.parametrize("bcl,bcr", [(N, NH), (N, DH), (D, NH), (D, DH)])
def test_pulse_equals_images_fp64(bcl, bcr):
    n, dx, c0 = 160, 1e-4, 1500.0
    L = (n - 0.5) * dx
    dt = 0.2 * dx / c0
    xs, sigma, m = 0.3 * L, 4 * dx, 1900                       # c0 t = 380 dx: both walls hit
    x = np.arange(n) * dx
    rl = 1.0 if bcl == N else -1.0
    rr = 1.0 if bcr == NH else -1.0

    def sources(jmax):
        js = range(-jmax, jmax + 1)
        return ([(xs + 2 * j * L, (rl * rr) ** abs(j)) for j in js] +
                [(-xs + 2 * j * L, rl * (rl * rr) ** abs(j)) for j in js])

    p0 = sum(s * np.exp(-0.5 * (x - c) ** 2 / sigma ** 2) for c, s in sources(2))
    case = workloads.Case("halfwall_pulse", (n,), ((bcl, bcr),), dx, dt, c0, m, p0, precision="fp64")
    print("halfwall pulse", bcl, bcr, flush=True)
    p, _ = run_gpu(case)
    reach = c0 * m * dt + 12 * sigma
    ref = sum(s * images.free_space_gaussian(np.abs(x - c), 1, 1.0, sigma, c0, dt, m)
              for c, s in sources(int(reach / (2 * L)) + 2))
    assert np.max(np.abs(p - ref)) < 1e-9


@pytest.mark.parametrize("seed,shape,bcs,prec,steps", [
    (21, (3, 5), ((N, DH), (D, NH)), "fp32", 30),        # minimal axes, fused path
    (22, (3,), ((D, NH),), "fp64", 30),                  # minimal 1D axis: one p sample, two u samples
    (23, (513, 20), ((D, DH), (N, N)), "fp32", 10),      # just above the fused limit: per-axis contractions
    (24, (1400,), ((N, NH),), "fp64", 10),               # 1D above the single-workgroup size: dense path
])
def test_edge_sizes(seed, shape, bcs, prec, steps):
    print("halfwall edge", shape, bcs, prec, flush=True)
    _check(_case(seed, shape, bcs, steps, prec))


def test_left_face_rejected():
    from paper_2005_00322_amd import Plan, PstdError
    with pytest.raises(PstdError):
        Plan((32, 32), 1e-4, 1e-8, 1500.0, ((NH, N), (N, N)), precision="fp32")
    with pytest.raises(PstdError):
        Plan((32, 32), 1e-4, 1e-8, 1500.0, ((P, NH), (N, N)), precision="fp32")
