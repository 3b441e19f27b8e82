"""Pins of the oracle's half-step-wall axes (groups III/IV of Table DTT_wavenumber_groups, types V-VIII):
a reflected pulse equals the sum of its image sources, energy is conserved, and the sequence lengths and
implied periods agree with the table."""
import numpy as np
import pytest

from oracle import images
from oracle import pstd

N, D, NH, DH = pstd.NEUMANN, pstd.DIRICHLET, pstd.NEUMANN_HALF, pstd.DIRICHLET_HALF
CASES = [(N, NH), (N, DH), (D, NH), (D, DH)]


@pytest.mark.parametrize("bcl,bcr", CASES)
def test_pulse_equals_images(bcl, bcr):
    """Walls on x = 0 and x = L = (n - 1/2) dx: the field is the free-space pulse plus its images at
    +-xs + 2jL, an image reflected in a Dirichlet wall changing sign."""
    n, dx, c0 = 160, 1e-4, 1500.0
    L = (n - 0.5) * dx
    dt = 0.2 * dx / c0
    xs, sigma = 0.3 * L, 4 * dx
    x = np.arange(n) * dx
    rl = 1.0 if bcl == N else -1.0
    rr = 1.0 if bcr == NH else -1.0
    def sources(jmax):
        js = range(-jmax, jmax + 1)
        return ([(xs + 2 * j * L, (rl * rr) ** abs(j)) for j in js] +
                [(-xs + 2 * j * L, rl * (rl * rr) ** abs(j)) for j in js])

    p0 = sum(s * np.exp(-0.5 * (x - c) ** 2 / sigma ** 2) for c, s in sources(2))
    prob = pstd.Problem((n,), ((bcl, bcr),), dx, dt, c0)
    for m in (1, 500, 1900):                                   # c0 t = 100 dx and 380 dx: both walls hit
        p, _ = prob.run(p0, m)
        reach = c0 * m * dt + 12 * sigma                       # images farther away have not arrived
        ref = sum(s * images.free_space_gaussian(np.abs(x - c), 1, 1.0, sigma, c0, dt, m)
                  for c, s in sources(int(reach / (2 * L)) + 2))
        assert np.max(np.abs(p - ref)) < 1e-9, m


@pytest.mark.parametrize("bcl,bcr", CASES)
def test_energy_and_shapes(bcl, bcr):
    rng = np.random.default_rng(7)
    shape, dx, c0 = (18, 15), 1e-4, 1500.0
    dt = 0.3 * dx / c0
    prob = pstd.Problem(shape, ((bcl, bcr), (D, N)), dx, dt, c0)
    assert prob.u_shape(0) == (18, 15) and prob.u_shape(1) == (18, 14)
    q = prob.project(rng.standard_normal(shape))
    u = prob.initial_velocity(q)
    energies = []
    for _ in range(60):
        q2, u2 = prob.step(q, u)
        energies.append(prob.energy(q, u, u2))
        q, u = q2, u2
    assert np.ptp(energies) < 1e-11 * abs(energies[0])


# Table DTT_wavenumber_groups: symmetry of p (whole-sample left, half-sample right) and of u, and the
# implied period of each type in terms of its own number of samples N.
TABLE = {(N, NH): ((2, -1), (2, 1)),     # p WSHS DCT-V M = 2N-1, u HAWA DST-VI M = 2N+1
         (N, DH): ((2, -1), (2, -1)),    # p WSHA DCT-VII 2N-1,   u HAWS DST-VIII 2N-1
         (D, NH): ((2, 1), (2, 1)),      # p WAHS DST-VII 2N+1,   u HSWA DCT-VIII 2N+1
         (D, DH): ((2, 1), (2, -1))}     # p WAHA DST-V 2N+1,     u HSWS DCT-VI 2N-1


@pytest.mark.parametrize("bcl,bcr", CASES)
@pytest.mark.parametrize("n", [3, 8, 21])
def test_lengths_and_periods(bcl, bcr, n):
    ax = pstd.HalfWallAxis(n, bcl, bcr, 1.0)
    (a1, b1), (a2, b2) = TABLE[(bcl, bcr)]
    Np, Nu = len(ax.k1), len(ax.k2)
    assert a1 * Np + b1 == ax.M == 2 * n - 1
    assert a2 * Nu + b2 == ax.M
    assert ax.periodic == ((bcl == N) == (bcr == NH))          # group III, else IV
    # div . grad maps every p mode to -k^2 times itself
    G, Dm = ax.grad_matrix(), ax.div_matrix()
    for m in range(Np):
        mode = np.zeros(n)
        mode[ax.p_lo:] = ax.T1inv[:, m]
        np.testing.assert_allclose(Dm @ (G @ mode), -ax.k1[m] ** 2 * mode, atol=1e-9 * max(1.0, ax.k1[m] ** 2))


def test_half_wall_is_a_right_face():
    with pytest.raises(ValueError):
        pstd.Problem((10,), ((NH, N),), 1e-4, 1e-8, 1500.0)
