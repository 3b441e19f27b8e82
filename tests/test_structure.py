"""Toeplitz-plus-Hankel form of the per-axis operators, as the library finds it on the host
(pstd_axis_operator_structure): every operator of every boundary family is rebuilt from its f, g and end
weights and compared with the FP64 matrix, entry by entry.  The split-bf16 contractions form their
operator slices from this form on the chip."""
import numpy as np
import pytest

from paper_2005_00322_amd.pstd import (DIRICHLET as D, DIRICHLET_HALF as DH, NEUMANN as N, NEUMANN_HALF as NH,
                                       PERIODIC as P, axis_operator, axis_operator_structure)

PAIRS = [(N, N), (D, D), (N, D), (D, N), (N, NH), (D, DH), (N, DH), (D, NH), (P, P)]


def _rebuild(f, g, w, R, C):
    r, c = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
    wr = np.ones(R)
    wr[0], wr[-1] = w[0], w[1]
    wc = np.ones(C)
    wc[0], wc[-1] = w[2], w[3]
    return wr[:, None] * wc[None, :] * (f[r - c + C - 1] + g[r + c])


@pytest.mark.parametrize("n", [7, 24, 97, 200, 385])
@pytest.mark.parametrize("pair", PAIRS)
def test_operators_rebuild_from_structure(n, pair):
    walls_on_nodes = pair[0] != P and pair[1] in (N, D)
    for which in range(6 if walls_on_nodes else 2):
        A = axis_operator(n, pair[0], pair[1], 1e-4, which)
        f, g, w, resid = axis_operator_structure(n, pair[0], pair[1], 1e-4, which)
        R, C = A.shape
        assert f.shape == g.shape == (R + C - 1,)
        err = np.abs(_rebuild(f, g, w, R, C) - A).max() / np.abs(A).max()
        assert err < 1e-11 and abs(err - resid) < 1e-13, (which, err, resid)


def test_end_weights_follow_the_walls():
    # a Neumann node counts once in the even extension (weight 1/2 on its column of G); a Dirichlet node
    # is held at zero (zero column of G, zero row of D); staggered points carry no weight
    n = 24
    assert list(axis_operator_structure(n, N, N, 1e-4, 0)[2]) == [1.0, 1.0, 0.5, 0.5]
    assert list(axis_operator_structure(n, D, D, 1e-4, 0)[2]) == [1.0, 1.0, 0.0, 0.0]
    assert list(axis_operator_structure(n, D, D, 1e-4, 1)[2]) == [0.0, 0.0, 1.0, 1.0]
    assert list(axis_operator_structure(n, N, D, 1e-4, 0)[2]) == [1.0, 1.0, 0.5, 0.0]
    assert list(axis_operator_structure(n, N, N, 1e-4, 1)[2]) == [1.0, 1.0, 1.0, 1.0]


def test_periodic_operators_are_toeplitz():
    # a circulant has no Hankel part: g is one constant per parity of r + c (the gauge freedom)
    for which in (0, 1):
        f, g, w, _ = axis_operator_structure(40, P, P, 1e-4, which)
        assert list(w) == [1.0, 1.0, 1.0, 1.0]
        scale = np.abs(f).max()
        for par in (0, 1):
            assert np.ptp(g[par::2]) < 1e-12 * scale


def test_gauge_keeps_parts_small():
    # f and g carry the least sum of squares: neither exceeds the operator's largest entry by much
    for pair in PAIRS:
        A = axis_operator(385, pair[0], pair[1], 1e-4, 0)
        f, g, _, _ = axis_operator_structure(385, pair[0], pair[1], 1e-4, 0)
        assert max(np.abs(f).max(), np.abs(g).max()) < 1.5 * np.abs(A).max()
