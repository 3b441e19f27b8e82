"""Pins of the oracle's time stepping (CPU only).

* A single standing mode of the box evolves as cos(m theta) cos(k x) with sin(theta/2) = c0 dt k / 2:
  a closed form that involves no transform (1D each boundary pair, 2D product mode).
* The discrete acoustic energy is conserved to rounding (1D/2D/3D, homogeneous and mapped c0).
* The transform-based modal closed form equals the stepped solution (both initial-velocity readings).
* The image-source solution with the leapfrog's dispersion relation (no transform at all) equals the
  stepped solution on the 1D Dirichlet workload (128 nodes, 1000 steps) and on a 2D mixed-wall box.
* §4.2's convergence study: at t = L/c0 with a centred Gaussian in a Neumann-Neumann box the error
  falls by ~16x per halving of CFL (every box mode then has omega t = pi n, so the leading phase
  error cancels), and reaches the quoted "0.1 %" level at modest CFL.
"""
import numpy as np
import pytest

import workloads
from oracle import images, pstd

N, D = pstd.NEUMANN, pstd.DIRICHLET
CASES = [(N, N), (N, D), (D, N), (D, D)]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("bc", CASES)
def test_standing_mode_1d(bc):
    n, dx, c0 = 41, 1e-4, 1500.0
    dt = 0.5 * dx / c0
    prob = pstd.Problem((n,), (bc,), dx, dt, c0)
    x = np.arange(n) * dx
    ax = prob.axes[0]
    for k in ax.k1[[0, 3, len(ax.k1) - 1]]:
        p0 = np.cos(k * x) if bc[0] == N else np.sin(k * x)
        m = 137
        p, _ = prob.run(p0, m)
        theta = 2 * np.arcsin(c0 * dt * k / 2)
        ref = prob.project(np.cos(m * theta) * p0)
        assert np.max(np.abs(p - ref)) < 1e-11


def test_standing_mode_2d():
    nx, ny, dx, c0 = 21, 17, 1e-4, 1500.0
    dt = 0.3 * dx / c0
    prob = pstd.Problem((nx, ny), ((D, N), (N, N)), dx, dt, c0)
    kx = prob.axes[0].k1[2]
    ky = prob.axes[1].k1[5]
    X, Y = np.meshgrid(np.arange(nx) * dx, np.arange(ny) * dx, indexing="ij")
    p0 = np.sin(kx * X) * np.cos(ky * Y)
    m = 250
    p, _ = prob.run(p0, m)
    theta = 2 * np.arcsin(c0 * dt * np.hypot(kx, ky) / 2)
    assert np.max(np.abs(p - np.cos(m * theta) * p0)) < 1e-11


@pytest.mark.parametrize("shape,bcs", [
    ((37,), ((N, D),)),
    ((19, 23), ((N, N), (D, N))),
    ((9, 11, 10), ((D, D), (N, D), (N, N))),
])
@pytest.mark.parametrize("mapped", [False, True])
def test_energy_conserved(shape, bcs, mapped):
    rng = np.random.default_rng(len(shape) * 7 + mapped)
    dx, c0 = 1e-4, 1500.0
    cmap = rng.uniform(1400, 1600, size=shape) if mapped else None
    dt = 0.2 * dx / 1600.0
    prob = pstd.Problem(shape, bcs, dx, dt, c0, c0_map=cmap)
    p = prob.project(rng.standard_normal(shape))
    u = prob.initial_velocity(p)
    E = []
    for _ in range(60):
        p2, u2 = prob.step(p, u)
        E.append(prob.energy(p, u, u2))
        p, u = p2, u2
    E = np.array(E)
    assert np.max(np.abs(E - E[0])) < 1e-12 * abs(E[0])


@pytest.mark.parametrize("u_mode", ["centred", "zero"])
@pytest.mark.parametrize("seed,ndim", [(0, 1), (1, 2), (2, 3), (3, 2)])
def test_modal_closed_form_matches_stepping(u_mode, seed, ndim):
    case = workloads.random_small_case(seed, ndim, max_n=24 if ndim == 3 else 40, steps=150)
    prob = pstd.Problem(case.shape, case.bcs, case.dx, case.dt, case.c0)
    p, _ = prob.run(case.p0, case.steps, u_mode=u_mode)
    ref = prob.modal_solution(case.p0, case.steps, u_mode=u_mode)
    assert _rel(p, ref) < 1e-11


def test_image_solution_1d_workload():
    case = workloads.pstd1d()
    prob = pstd.Problem(case.shape, case.bcs, case.dx, case.dt, case.c0)
    c, s = case.extra["centre"], case.extra["sigma"]
    p0 = images.image_summed_gaussian(case.shape, case.bcs, case.dx, c, 1.0, s)
    p, _ = prob.run(p0, case.steps)
    ref = images.image_solution(case.shape, case.bcs, case.dx, case.c0, case.dt, case.steps, c, 1.0, s)
    assert _rel(p, ref) < 1e-11
    # against omega = c0 k the difference is the time-dispersion error, O(CFL^2)
    cont = images.image_solution(case.shape, case.bcs, case.dx, case.c0, case.dt, case.steps, c, 1.0, s,
                                 u_mode="continuous")
    assert 1e-3 < _rel(p, cont) < 2e-2


@pytest.mark.parametrize("u_mode", ["centred", "zero"])
def test_image_solution_2d_mixed_walls(u_mode):
    shape, dx, c0 = (48, 40), 1e-4, 1500.0
    bcs = ((D, N), (N, D))
    dt = 0.3 * dx / c0
    centre, sigma = (20 * dx, 14 * dx), 3.5 * dx
    prob = pstd.Problem(shape, bcs, dx, dt, c0)
    p0 = images.image_summed_gaussian(shape, bcs, dx, centre, 1.0, sigma)
    m = 160                                  # c0 t = 48 dx: several wall reflections, both corners
    p, _ = prob.run(p0, m, u_mode=u_mode)
    ref = images.image_solution(shape, bcs, dx, c0, dt, m, centre, 1.0, sigma, u_mode=u_mode)
    assert _rel(p, ref) < 1e-9


def test_convergence_with_cfl():
    n, dx, c0 = 129, 1e-4, 1500.0
    L = (n - 1) * dx
    errs = []
    for cfl in (0.5, 0.25, 0.125, 0.0625):
        dt = cfl * dx / c0
        steps = int(round(L / (c0 * dt)))
        prob = pstd.Problem((n,), ((N, N),), dx, dt, c0)
        p0 = workloads.gaussian((n,), dx, (L / 2,), 4 * dx)
        p = prob.modal_solution(p0, steps)
        errs.append(np.max(np.abs(p - p0)) / np.max(np.abs(p0)))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 14.0) and np.all(ratios < 17.0)
    assert errs[1] < 1e-3                    # "0.1 %" reached at CFL 0.25


def test_convergence_stepping_agrees_with_closed_form():
    n, dx, c0, cfl = 129, 1e-4, 1500.0, 0.25
    L = (n - 1) * dx
    dt = cfl * dx / c0
    steps = int(round(L / (c0 * dt)))
    prob = pstd.Problem((n,), ((N, N),), dx, dt, c0)
    p0 = workloads.gaussian((n,), dx, (L / 2,), 4 * dx)
    p, _ = prob.run(p0, steps)
    assert _rel(p, prob.modal_solution(p0, steps)) < 1e-11
