"""Pins of the oracle's collocated differentiation (§3.3) and staggered interpolation (§3.4).

Every basis function of an axis's pressure space (whole-sample symmetry of its boundary pair) and of
its velocity space (half-sample) is a trigonometric mode whose derivative and half-step shift are known
in closed form; the four operators must reproduce those values exactly (to rounding) on every mode, which
fixes each operator completely on its space.
"""
import numpy as np
import pytest

from oracle import pstd as o

N, D = o.NEUMANN, o.DIRICHLET
CASES = [(N, N), (N, D), (D, N), (D, D)]


def modes(n, bcl, bcr, dx):
    """(p modes, u modes): lists of (f, f') callables spanning the p nodes and the staggered points."""
    L = (n - 1) * dx
    anti = bcl != bcr                                   # mixed walls: k = pi (m + 1/2) / L
    ks = lambda ms: [np.pi * (m + (0.5 if anti else 0.0)) / L for m in ms]
    cos = lambda k: (lambda x: np.cos(k * x), lambda x: -k * np.sin(k * x))
    sin = lambda k: (lambda x: np.sin(k * x), lambda x: k * np.cos(k * x))
    if (bcl, bcr) == (N, N):
        return [cos(k) for k in ks(range(0, n))], [sin(k) for k in ks(range(1, n))]
    if (bcl, bcr) == (D, D):
        return [sin(k) for k in ks(range(1, n - 1))], [cos(k) for k in ks(range(0, n - 1))]
    if (bcl, bcr) == (N, D):
        return [cos(k) for k in ks(range(0, n - 1))], [sin(k) for k in ks(range(0, n - 1))]
    return [sin(k) for k in ks(range(0, n - 1))], [cos(k) for k in ks(range(0, n - 1))]


@pytest.mark.parametrize("bcl,bcr", CASES)
@pytest.mark.parametrize("n", [5, 9, 16, 17])
def test_every_mode_exact(bcl, bcr, n):
    dx = 0.37
    ax = o.Axis(n, bcl, bcr, dx)
    xn = np.arange(n) * dx
    xh = (np.arange(n - 1) + 0.5) * dx
    pm, um = modes(n, bcl, bcr, dx)
    kmax = np.pi / dx
    for f, df in pm:
        p = f(xn)
        assert np.max(np.abs(ax.collocated_grad_p(p) - df(xn))) < 1e-11 * kmax
        assert np.max(np.abs(ax.interp_p_to_u(p) - f(xh))) < 1e-11
    for f, df in um:
        u = f(xh)
        assert np.max(np.abs(ax.collocated_grad_u(u) - df(xh))) < 1e-11 * kmax
        assert np.max(np.abs(ax.interp_u_to_p(u) - f(xn))) < 1e-11


@pytest.mark.parametrize("bcl,bcr", CASES)
def test_mode_counts_span_the_spaces(bcl, bcr):
    """The modes used above are as many as the unknowns, so exactness on them fixes the operators."""
    n = 12
    ax = o.Axis(n, bcl, bcr, 1.0)
    pm, um = modes(n, bcl, bcr, 1.0)
    assert len(pm) == ax.p_hi - ax.p_lo + 1
    assert len(um) == n - 1
    xn, xh = np.arange(n), np.arange(n - 1) + 0.5
    P = np.array([f(xn)[ax.p_lo:ax.p_hi + 1] for f, _ in pm])
    U = np.array([f(xh) for f, _ in um])
    assert np.linalg.matrix_rank(P) == len(pm) and np.linalg.matrix_rank(U) == len(um)


@pytest.mark.parametrize("bcl,bcr", CASES)
@pytest.mark.parametrize("n", [6, 11])
def test_shapes_and_staggered_compositions(bcl, bcr, n):
    """Shapes of the four matrices, and the collocated derivatives equal the staggered derivative of
    Eq. (dtt_pstd_solution) followed by a half-step shift back: on the nodes interp_u_to_p . grad, on
    the staggered points interp_p_to_u . div (every mode, including the Nyquist ones that vanish)."""
    ax = o.Axis(n, bcl, bcr, 0.5)
    shapes = {2: (n, n), 3: (n - 1, n - 1), 4: (n - 1, n), 5: (n, n - 1)}
    for w, shp in shapes.items():
        assert ax.resample_matrix(w).shape == shp
    np.testing.assert_allclose(ax.resample_matrix(2), ax.resample_matrix(5) @ ax.grad_matrix(), atol=1e-11)
    np.testing.assert_allclose(ax.resample_matrix(3), ax.resample_matrix(4) @ ax.div_matrix(), atol=1e-11)
