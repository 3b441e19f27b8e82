"""Pins of the periodic (Fourier) axis of the oracle (Eq. (fourier_pstd_solution), §2; CPU only).

* Staggered derivatives of single Fourier modes are exact: grad of sin(2 pi q x / L) on the nodes is
  (2 pi q / L) cos(2 pi q (x + dx/2) / L) on the staggered points, div maps back likewise; the Nyquist
  mode (-1)^j of an even axis differentiates like its band-limited interpolant cos(pi x / dx).
* div(grad) has the eigenvalues -k^2 on the Fourier modes, and W div = -grad^T (so the staggered step
  conserves the discrete energy), checked as matrices.
* In a 1D periodic box a band-limited Gaussian pulse equals the sum over its periodic images of the
  free-space solution of the same leapfrog (images.free_space_gaussian), long after it has wrapped.
* Shifting the initial field by whole nodes shifts the solution (translation invariance), and the
  discrete energy is conserved in a box with a periodic and a wall-bounded axis.
"""
import numpy as np
import pytest

from oracle import images, pstd

P, N, D = pstd.PERIODIC, pstd.NEUMANN, pstd.DIRICHLET


@pytest.mark.parametrize("n", [16, 17, 30])
def test_modes_differentiate_exactly(n):
    dx = 1e-4
    ax = pstd.PeriodicAxis(n, dx)
    L = n * dx
    x = np.arange(n) * dx
    for q in range(1, (n - 1) // 2 + 1):
        kq = 2 * np.pi * q / L
        g = ax.grad(np.sin(kq * x))
        assert np.max(np.abs(g - kq * np.cos(kq * (x + dx / 2)))) < 1e-9 * kq
        d = ax.div(np.cos(kq * (x + dx / 2)))
        assert np.max(np.abs(d + kq * np.sin(kq * x))) < 1e-9 * kq
    if n % 2 == 0:
        g = ax.grad((-1.0) ** np.arange(n))
        ref = -(np.pi / dx) * np.sin(np.pi * (np.arange(n) + 0.5))
        assert np.max(np.abs(g - ref)) < 1e-9 * np.pi / dx


@pytest.mark.parametrize("n", [12, 13])
def test_operator_structure(n):
    dx = 2e-4
    ax = pstd.PeriodicAxis(n, dx)
    G, Dm = ax.grad_matrix(), ax.div_matrix()
    assert np.allclose(Dm, -G.T, atol=1e-8 / dx)             # W = identity on a periodic axis
    ev = np.sort(np.linalg.eigvalsh(0.5 * ((Dm @ G) + (Dm @ G).T)))
    m = np.fft.fftfreq(n) * n
    ref = np.sort(-(2 * np.pi * m / (n * dx)) ** 2)
    assert np.allclose(ev, ref, rtol=1e-9, atol=1e-6 / dx ** 2)


def test_pulse_equals_periodic_images():
    n, dx, c0 = 200, 1e-4, 1500.0
    L = n * dx
    dt = 0.2 * dx / c0
    xs, sigma = 0.37 * L, 4 * dx
    x = np.arange(n) * dx
    prob = pstd.Problem((n,), ((P, P),), dx, dt, c0)
    for m in (300, 1300, 2600):                                # c0 t = 60, 260, 520 dx: wrapped twice
        p0 = sum(np.exp(-0.5 * (x - xs - j * L) ** 2 / sigma ** 2) for j in range(-2, 3))
        p, _ = prob.run(p0, m)
        reach = c0 * m * dt + 12 * sigma
        js = range(-int(reach / L) - 2, int(reach / L) + 3)
        ref = sum(images.free_space_gaussian(np.abs(x - xs - j * L), 1, 1.0, sigma, c0, dt, m) for j in js)
        assert np.max(np.abs(p - ref)) < 1e-10


def test_translation_and_energy():
    rng = np.random.default_rng(4)
    shape, dx, c0 = (20, 14), 1e-4, 1500.0
    dt = 0.3 * dx / c0
    prob = pstd.Problem(shape, ((P, P), (N, D)), dx, dt, c0)
    p0 = prob.project(rng.standard_normal(shape))
    p, _ = prob.run(p0, 40)
    ps, _ = prob.run(np.roll(p0, 3, axis=0), 40)
    assert np.max(np.abs(ps - np.roll(p, 3, axis=0))) < 1e-12 * np.max(np.abs(p))
    u = prob.initial_velocity(p0)
    q = p0
    energies = []
    for _ in range(60):
        q2, u2 = prob.step(q, u)
        energies.append(prob.energy(q, u, u2))
        q, u = q2, u2
    assert np.ptp(energies) < 1e-11 * abs(energies[0])
    assert prob.u_shape(0) == (20, 14) and prob.u_shape(1) == (20, 13)


def test_periodic_needs_both_faces():
    with pytest.raises(ValueError):
        pstd.Problem((10, 10), ((P, N), (N, N)), 1e-4, 1e-8, 1500.0)
